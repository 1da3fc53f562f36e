"""Discrete Green's function G^{h=1} of a Mehrstellen Laplacian
(paper sec. 2, eq. dgf; construction in appendix A.1).

G^{h=1} satisfies (L G)[g] = delta_0[g] and behaves like -1/(4 pi |g|) at
infinity.  The paper approximates it on D = [-Z, Z]^3 by solving the
inhomogeneous Dirichlet problem on the larger cube [-zeta Z, zeta Z]^3
(zeta = 2) with the continuous Green's function -1/(4 pi |g|) imposed on the
outer layer, in residual-correction form, by discrete sine transforms, and
restricting the result to D.  The paper uses Z >= 128 and zeta = 2; this
oracle takes Z as a parameter (default 128) and fixes zeta = 2.
"""
import numpy as np
import scipy.fft as sfft

from .stencils import apply_laplacian, symbol


def continuous_green(gz, gy, gx):
    """G(x) = -1/(4 pi |x|) (sec. 1, eq. potential); undefined at 0."""
    return -1.0 / (4.0 * np.pi * np.sqrt(gz * gz + gy * gy + gx * gx))


def dgf(Q, Z=128, workers=None):
    """G^{h=1} on [-Z, Z]^3 as an array of shape (2Z+1,)*3, centre at [Z,Z,Z].

    Steps (appendix A.1):
      1. L = 2Z; the big cube is [-L, L]^3, its interior [-L+1, L-1]^3.
      2. w = G(g) on the outer layer |g|_inf = L, 0 elsewhere.
      3. u solves L u = delta - L w in the interior with u = 0 on the layer
         (residual-correction form), by the 3-D DST-I whose modes
         sin(pi k (g+L) / 2L) diagonalise the stencil with eigenvalue
         symbol(cos(pi k0/2L), cos(pi k1/2L), cos(pi k2/2L)).
      4. G = u + w; restrict to [-Z, Z]^3 (where w = 0).
    """
    L = 2 * Z
    size = 2 * L + 1
    ax = np.arange(-L, L + 1, dtype=np.float64)
    # w on the outer layer: the six faces of the big cube (|g|_inf = L never
    # meets 0).  L w vanishes except on the interior layer next to the outer
    # layer, so it is formed slab by slab: a slab of three node layers at a
    # face holds the whole stencil of every interior node next to that face.
    rhs = np.zeros((size - 2,) * 3)
    on_edge = np.abs(ax) == L
    for side in (0, 1):
        g0 = ax[-3:] if side else ax[:3]
        g3 = continuous_green(g0[:, None, None], ax[None, :, None], ax[None, None, :])
        layer = (np.abs(g0) == L)[:, None, None] | on_edge[None, :, None] | on_edge[None, None, :]
        slab = np.where(layer, g3, 0.0)
        lap = -apply_laplacian(slab, Q)[0]           # the interior layer next to this face
        for d in range(3):                             # w is symmetric under axis permutations
            idx = [slice(None)] * 3
            idx[d] = -1 if side else 0
            rhs[tuple(idx)] = lap
    rhs[L - 1, L - 1, L - 1] += 1.0         # delta at the origin
    m = np.arange(1, 2 * L, dtype=np.float64)
    c = np.cos(np.pi * m / (2 * L))
    lam = symbol(Q, c[:, None, None], c[None, :, None], c[None, None, :])
    uh = sfft.dstn(rhs, type=1, norm="ortho", workers=workers)
    del rhs
    uh /= lam
    del lam
    u = sfft.idstn(uh, type=1, norm="ortho", workers=workers)
    del uh
    # interior index of g is g + L - 1
    lo = L - 1 - Z
    return np.ascontiguousarray(u[lo:lo + 2 * Z + 1, lo:lo + 2 * Z + 1, lo:lo + 2 * Z + 1])


_cache = {}


def dgf_cached(Q, Z=128):
    """Memoised dgf(Q, Z) for the lifetime of the process."""
    key = (Q, Z)
    if key not in _cache:
        _cache[key] = dgf(Q, Z)
    return _cache[key]
