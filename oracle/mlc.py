"""The fully discrete two-level Method of Local Corrections
(paper sec. 4.1, steps 1-3, with the Mehrstellen correction at the end).

Conventions
  * f is given on the (N+1)^3 fine nodes of [0, N]^3 (array axes 0, 1, 2),
    h = 1/N by default, and must vanish on the outer boundary nodes
    (the support of f lies inside the domain, sec. 4).
  * Patches Omega_i = n i + [0, n]^3 (node-centred, face-sharing).
  * d_alpha = ceil((alpha-1) n / 2), d_beta = ceil((beta-1) n / 2);
    Omega_{i,alpha} = G(Omega_i, d_alpha), Omega_{i,beta} = G(Omega_i, d_beta).
  * Local fields phi_i are evaluated on E_i = G(Omega_{i,alpha}, Nref b)
    (sec. 4.1 eq. initiallocalproblemsmlcII).
  * Coarse node c is the fine node Nref c; H = Nref h.

Readings of the paper used here (see the module docstrings of legendre and
interp for the other two):
  * d_alpha and d_beta must be multiples of Nref so that the localisation
    regions are coarse-aligned (the paper's settings all are).
  * F^{i,H} inner part lives on C(Omega_{i,alpha}) itself (sec. 4.1 eq. FDLD).
  * The coarse right-hand side is supported on the union of C(Omega_{i,beta})
    and phi^H is needed on [-b, N/Nref + b]^3 (the interpolation stencils of
    the skeleton nodes of [0, N]^3).
  * The final correction adds C2 h^2 f with C2 = 1/12 for both stencils
    (sec. 4.1 eq. mcapplicationfulldiscr); the sign of the defining relation
    is taken from sec. 2 eq. msCorr4.
"""
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

from . import convolution as conv
from . import legendre as leg
from .geometry import NREF, coarsen, grow, margin, patch_box, patch_indices
from .interp import lagrange_weights, normal_axis, stencil
from .stencils import C2, apply_laplacian, stencil_b, symbol


@dataclass(frozen=True)
class Params:
    N: int              # cells per axis of the fine grid
    n: int              # cells per patch edge
    alpha: float        # inner localisation radius (units of R = n h / 2)
    beta: float         # outer localisation radius
    P: int              # Legendre truncation: modes with |p|_1 < P
    Q: int              # 4 -> L19, 6 -> L27
    b: int = 0          # interpolation stencil radius; 0 -> Q/2
    h: float = 0.0      # mesh spacing; 0 -> 1/N
    Z: int = 128        # DGF table half-width

    @property
    def bb(self):
        return self.b if self.b else self.Q // 2

    @property
    def hh(self):
        return self.h if self.h else 1.0 / self.N

    @property
    def H(self):
        return NREF * self.hh

    @property
    def R(self):
        return self.n * self.hh / 2.0

    @property
    def d_alpha(self):
        return margin(self.alpha, self.n)

    @property
    def d_beta(self):
        return margin(self.beta, self.n)

    @property
    def e(self):
        """half-margin of E_i = G(Omega_{i,alpha}, Nref b) around Omega_i"""
        return self.d_alpha + NREF * self.bb

    @property
    def K(self):
        return self.P * (self.P + 1) * (self.P + 2) // 6

    def check(self):
        if self.N % self.n or self.n % NREF or self.n < 8:
            raise ValueError("need N % n == 0, n % 4 == 0, n >= 8")
        if self.alpha < 1 or self.beta < self.alpha:
            raise ValueError("need 1 <= alpha <= beta")
        if self.d_alpha % NREF or self.d_beta % NREF:
            raise ValueError("localisation margins must be multiples of Nref")
        if self.Q not in (4, 6):
            raise ValueError("Q must be 4 or 6")


def chi_1d(n):
    """Per-axis factor of the discrete characteristic function of a patch:
    1/2 at both ends, 1 inside (sec. 4: 1/8 corners, 1/4 edges, 1/2 faces)."""
    w = np.ones(n + 1)
    w[0] = w[-1] = 0.5
    return w


def patch_charge(f, n, i):
    """f^{i,h} = chi_{Omega_i} f on the (n+1)^3 patch nodes (sec. 4)."""
    lo = n * np.asarray(i)
    sub = f[lo[0]:lo[0] + n + 1, lo[1]:lo[1] + n + 1, lo[2]:lo[2] + n + 1]
    w = chi_1d(n)
    return sub * (w[:, None, None] * w[None, :, None] * w[None, None, :])


def local_field(G1, prm, q, mode="fft", cache=None):
    """phi_i = G^h * f^{i,h} on E_i (sec. 4.1 step 1), as an array over the
    relative box [-e, n+e]^3 of the patch."""
    e, n = prm.e, prm.n
    lo, hi = np.full(3, -e), np.full(3, n + e)
    if mode == "direct":
        out = conv.conv_direct(G1, prm.Z, q, lo, hi)
    else:
        out = conv.conv_hockney(G1, prm.Z, q, lo, hi, kernel_cache=cache)
    return prm.hh ** 2 * out


def coarse_laplacian_of_samples(phi_fine, Q, H):
    """Delta^H of the coarse samples phi[Nref c] (operators on finer data act
    by sampling, sec. 2).  phi_fine must start on a coarse node; the result
    covers the coarse nodes with a full stencil."""
    return apply_laplacian(phi_fine[::NREF, ::NREF, ::NREF], Q, H)


def far_field_tables(G1, prm, mode="fft"):
    """Fields of the Legendre modes of a unit patch placed at i = 0
    (sec. 4.1, 'can be computed once and stored'):
        Phi_p = G^h * (chi_{Omega_0} Q^p)   on G(Omega_{0,beta}, Nref b),
        T_p   = Delta^H Phi_p               on C(Omega_{0,beta}).
    Returns (Phi, T, phi_lo, T_lo) with arrays of shape (K, ...), and the
    relative low corners of their boxes."""
    n, P = prm.n, prm.P
    eb = prm.d_beta + NREF * prm.bb
    w = chi_1d(n)
    chi = w[:, None, None] * w[None, :, None] * w[None, None, :]
    B = leg.basis_on_patch(n, P) * prm.R ** -1.5
    lo, hi = np.full(3, -eb), np.full(3, n + eb)
    Phi = []
    cache = {}
    for k in range(len(B)):
        q = chi * B[k]
        if mode == "direct":
            Phi.append(prm.hh ** 2 * conv.conv_direct(G1, prm.Z, q, lo, hi))
        else:
            Phi.append(prm.hh ** 2 * conv.conv_hockney(G1, prm.Z, q, lo, hi, kernel_cache=cache))
    Phi = np.stack(Phi)
    # coarse samples start at -eb (a coarse node); the Laplacian drops one
    # coarse layer, leaving [-eb/4 + 1, (n+eb)/4 - 1] which contains
    # C(Omega_{0,beta}) = [-d_beta/4, (n+d_beta)/4] when b >= 1.
    T = np.stack([coarse_laplacian_of_samples(Phi[k], prm.Q, prm.H) for k in range(len(B))])
    T_lo = -eb // NREF + 1
    cb_lo, cb_hi = -prm.d_beta // NREF, (n + prm.d_beta) // NREF
    T = T[:, cb_lo - T_lo:cb_hi - T_lo + 1, cb_lo - T_lo:cb_hi - T_lo + 1, cb_lo - T_lo:cb_hi - T_lo + 1]
    return Phi, T, -eb, cb_lo


def coarse_boxes(prm):
    """(S_lo, S_hi): support box of F^H; (O_lo, O_hi): where phi^H is kept."""
    S_lo = -prm.d_beta // NREF
    S_hi = (prm.N + prm.d_beta) // NREF
    O_lo = -prm.bb
    O_hi = prm.N // NREF + prm.bb
    return S_lo, S_hi, O_lo, O_hi


def interp_matrix(b, fine_lo, fine_hi, coarse_lo, coarse_hi):
    """1-D matrix of the coplanar interpolation along one in-plane axis:
    row x (fine coordinate) holds the Lagrange weights of the coarse nodes
    floor(x/4) - b .. floor(x/4) + b + 1; a row with theta = 0 has the single
    weight 1.  Columns are coarse coordinates coarse_lo..coarse_hi."""
    xs = np.arange(fine_lo, fine_hi + 1)
    A = np.zeros((len(xs), coarse_hi - coarse_lo + 1))
    for r, x in enumerate(xs):
        U0 = x // NREF
        th = (x - NREF * U0) / NREF
        if th == 0.0:
            A[r, U0 - coarse_lo] = 1.0
            continue
        w = lagrange_weights(b, th)
        cols = U0 + np.arange(-b, b + 2) - coarse_lo
        if cols[0] < 0 or cols[-1] >= A.shape[1]:
            raise ValueError("interpolation stencil leaves the coarse data")
        A[r, cols] = w
    return A


def skeleton_mask(N, n):
    ax = (np.arange(N + 1) % n) == 0
    return ax[:, None, None] | ax[None, :, None] | ax[None, None, :]


def _plane_iter(d_lo, d_hi, n):
    """Plane coordinates P in [d_lo, d_hi] with P % n == 0."""
    start = -(-d_lo // n) * n
    return range(start, d_hi + 1, n)


def _canonical_keep(coords_a, coords_b, d, a, bax, n, shape):
    """Mask over a plane of normal d keeping only nodes whose canonical
    normal axis is d (no axis below d divisible by n)."""
    keep = np.ones(shape, dtype=bool)
    for ax, cs, sl in ((a, coords_a, (slice(None), None)), (bax, coords_b, (None, slice(None)))):
        if ax < d:
            keep &= ~((cs % n) == 0)[sl]
    return keep


def _plane_views(d):
    a0, a1 = [a for a in range(3) if a != d]
    return a0, a1


def _take_plane(arr, d, idx):
    return np.take(arr, idx, axis=d)


def plan_tables(G1, prm, conv_mode="fft"):
    """The per-problem-class tables of the Legendre far field (sec. 4.1:
    computed once and stored): far_field_tables and, for the regrouped
    boundary values, _annulus_plane_tables.  None when beta == alpha."""
    if not prm.beta > prm.alpha:
        return None
    Phi, T, Phi_lo, T_lo = far_field_tables(G1, prm, mode=conv_mode)
    return dict(Phi=Phi, T=T, Phi_lo=Phi_lo, T_lo=T_lo, planes=_annulus_plane_tables(Phi, Phi_lo, prm))


def mlc_solve(f, prm, G1=None, conv_mode="fft", bc_mode="by_patch", keep=False, on_local=None, tables=None,
              moments_fn=None, coarse_fn=None, correct=True):
    """Two-level MLC (sec. 4.1).  Returns phi on all (N+1)^3 nodes and, if
    keep, a dict of intermediates: moments, FH, phiH, phiB (full grid,
    meaningful on skeleton nodes), and the per-patch local fields (only for
    bc_mode='literal').  on_local, if given, is called as
    on_local(patch_number, i, phi_i) with each local field on E_i as soon as
    it is computed (read only; it lets a caller inspect every patch's field
    without keeping them all).  tables, if given, is plan_tables(G1, prm)
    built beforehand (the same values the solve would build).  moments_fn,
    if given, returns the Legendre coefficients of patch i (moments_fn(i)),
    e.g. legendre.moments_gauss for a charge given analytically (sec. 4.1
    step 1); otherwise they come from the node values by Boole's rule.
    coarse_fn, if given, replaces the coarse convolution of step 2:
    coarse_fn(FH, S_lo, O_lo, O_hi) returns phi^H on [O_lo, O_hi]^3 (the
    multilevel method solves the coarse charge by MLC one level up, sec. 5).
    correct=False leaves out the final C2 h^2 f (the charge is then a
    modified right-hand side, see mlc_solve_sixth)."""
    from .dgf import dgf_cached
    prm.check()
    N, n, Q, b = prm.N, prm.n, prm.Q, prm.bb
    h, H, R = prm.hh, prm.H, prm.R
    da, db, e = prm.d_alpha, prm.d_beta, prm.e
    if G1 is None:
        G1 = dgf_cached(Q, prm.Z)
    if f.shape != (N + 1,) * 3:
        raise ValueError("f must have shape (N+1,)*3")
    patches = patch_indices(N, n)
    S_lo, S_hi, O_lo, O_hi = coarse_boxes(prm)
    FH = np.zeros((S_hi - S_lo + 1,) * 3)
    K = prm.K
    moments = np.zeros((len(patches), K))
    annulus = prm.beta > prm.alpha
    if annulus:
        if tables is None:
            Phi, T, Phi_lo, T_lo = far_field_tables(G1, prm, mode=conv_mode)
            tabs = _annulus_plane_tables(Phi, Phi_lo, prm) if bc_mode != "literal" else None
        else:
            Phi, T, Phi_lo, T_lo, tabs = (tables[k] for k in ("Phi", "T", "Phi_lo", "T_lo", "planes"))
    cache = {}
    skel = skeleton_mask(N, n)
    accum = np.zeros((N + 1,) * 3)        # sum of (loc - I(loc)) per node
    fields = {} if bc_mode == "literal" else None

    # ---- step 1: local convolutions, moments, local coarse charges ----
    for pi, i in enumerate(patches):
        lo = n * i
        q = patch_charge(f, n, i)
        phi_i = local_field(G1, prm, q, conv_mode, cache)          # on [lo-e, lo+n+e]
        fpatch = f[lo[0]:lo[0] + n + 1, lo[1]:lo[1] + n + 1, lo[2]:lo[2] + n + 1]
        c = leg.moments(fpatch, n, prm.P, R) if moments_fn is None else moments_fn(i)
        moments[pi] = c
        if on_local is not None:
            on_local(pi, i, phi_i)
        # inner part: Delta^H phi_i on C(Omega_{i,alpha})
        lap = coarse_laplacian_of_samples(phi_i, Q, H)              # coarse nodes from (lo-e)/4+1
        lap_lo = (lo - e) // NREF + 1
        ca_lo = (lo - da) // NREF
        ca_hi = (lo + n + da) // NREF
        sl = tuple(slice(ca_lo[d] - lap_lo[d], ca_hi[d] - lap_lo[d] + 1) for d in range(3))
        tgt = tuple(slice(ca_lo[d] - S_lo, ca_hi[d] - S_lo + 1) for d in range(3))
        FH[tgt] += lap[sl]
        # annulus part: sum_p c_p T_p on C(Omega_{i,beta}) \ C(Omega_{i,alpha})
        if annulus:
            cb_lo = (lo - db) // NREF
            cb_hi = (lo + n + db) // NREF
            ann = np.einsum("k,kabc->abc", c, T)                    # on [cb_lo, cb_hi] rel. patch
            inner = np.zeros(ann.shape, dtype=bool)
            o = ca_lo - cb_lo
            inner[o[0]:o[0] + ca_hi[0] - ca_lo[0] + 1,
                  o[1]:o[1] + ca_hi[1] - ca_lo[1] + 1,
                  o[2]:o[2] + ca_hi[2] - ca_lo[2] + 1] = True
            ann[inner] = 0.0
            tgt = tuple(slice(cb_lo[d] - S_lo, cb_hi[d] - S_lo + 1) for d in range(3))
            FH[tgt] += ann
        if bc_mode == "literal":
            fields[tuple(i)] = phi_i
        else:
            _accumulate_local(accum, phi_i, lo, prm)
            if annulus:
                _accumulate_annulus(accum, c, tabs, lo, prm)

    # ---- step 2: coarse solve phi^H = G^H * F^H on [O_lo, O_hi] ----
    if coarse_fn is None:
        phiH = H ** 2 * conv.conv_hockney(G1, prm.Z, FH, np.full(3, O_lo - S_lo), np.full(3, O_hi - S_lo))
    else:
        phiH = coarse_fn(FH, S_lo, O_lo, O_hi)

    # ---- step 3: boundary values on the skeleton ----
    if bc_mode == "literal":
        phiB = _boundary_literal(fields, moments, patches, Phi if annulus else None,
                                 Phi_lo if annulus else 0, phiH, O_lo, prm)
    else:
        phiB = accum + _interp_coarse_everywhere(phiH, O_lo, prm)
    phiB = np.where(skel, phiB, 0.0)

    # ---- Dirichlet solves on each patch, then the Mehrstellen correction ----
    phit = phiB.copy()
    for i in patches:
        lo = n * i
        sl = tuple(slice(lo[d], lo[d] + n + 1) for d in range(3))
        phit[sl][1:-1, 1:-1, 1:-1] = dirichlet_solve(phiB[sl], f[sl], Q, h)
    phi = phit + C2 * h * h * f if correct else phit.copy()
    if not keep:
        return phi
    out = dict(moments=moments, FH=FH, S_lo=S_lo, phiH=phiH, O_lo=O_lo, phiB=phiB, phitilde=phit)
    if fields is not None:
        out["fields"] = fields
    return phi, out


def dirichlet_solve(bvals, fpatch, Q, h):
    """Interior values of the discrete Dirichlet problem on one patch
    (sec. 4.1 eq. last_step_fulldiscr): Delta^h u = f at the interior nodes,
    u = bvals on the patch boundary.  The boundary terms move to the right
    side; the zero-boundary problem is diagonal in the DST-I basis of
    length n-1 (eigenvalues symbol(cos(pi k / n), ...))."""
    n = bvals.shape[0] - 1
    bnd = bvals.copy()
    bnd[1:-1, 1:-1, 1:-1] = 0.0
    rhs = h * h * fpatch[1:-1, 1:-1, 1:-1] - apply_laplacian(bnd, Q)
    cs = np.cos(np.pi * np.arange(1, n) / n)
    lam = symbol(Q, cs[:, None, None], cs[None, :, None], cs[None, None, :])
    return sfft.idstn(sfft.dstn(rhs, type=1, norm="ortho") / lam, type=1, norm="ortho")


def _accumulate_local(accum, phi_i, lo, prm):
    """accum[g] += phi_i[g] - I(phi_i)(g) for the skeleton nodes g of
    Omega_{i,alpha} inside [0, N]^3 (each node once, on its canonical plane).
    By linearity of I this is patch i's share of loc_g(g) - I(loc_g)(g) over
    the patches with g in Omega_{i,alpha}."""
    N, n, b, da, e = prm.N, prm.n, prm.bb, prm.d_alpha, prm.e
    a_lo = np.maximum(lo - da, 0)
    a_hi = np.minimum(lo + n + da, N)
    E_lo = lo - e
    for d in range(3):
        a0, a1 = _plane_views(d)
        A0 = interp_matrix(b, a_lo[a0], a_hi[a0], E_lo[a0] // NREF, (lo[a0] + n + e) // NREF)
        A1 = interp_matrix(b, a_lo[a1], a_hi[a1], E_lo[a1] // NREF, (lo[a1] + n + e) // NREF)
        x0 = np.arange(a_lo[a0], a_hi[a0] + 1)
        x1 = np.arange(a_lo[a1], a_hi[a1] + 1)
        keep = _canonical_keep(x0, x1, d, a0, a1, n, (len(x0), len(x1)))
        for P in _plane_iter(a_lo[d], a_hi[d], n):
            plane = _take_plane(phi_i, d, P - E_lo[d])             # axes (a0, a1) over E_i
            fine = plane[x0[0] - E_lo[a0]:x0[-1] - E_lo[a0] + 1, x1[0] - E_lo[a1]:x1[-1] - E_lo[a1] + 1]
            coarse = plane[::NREF, ::NREF]
            val = fine - A0 @ coarse @ A1.T
            idx = [None, None, None]
            idx[d] = P
            idx[a0] = slice(x0[0], x0[-1] + 1)
            idx[a1] = slice(x1[0], x1[-1] + 1)
            view = accum[tuple(idx)]
            view += np.where(keep, val, 0.0)


def _annulus_plane_tables(Phi, Phi_lo, prm):
    """D_p = Phi_p - I(Phi_p) on every skeleton plane of Omega_{0,beta}
    (relative coordinates), keyed by (d, P)."""
    n, b, db = prm.n, prm.bb, prm.d_beta
    eb = db + NREF * b
    out = {}
    for d in range(3):
        a0, a1 = _plane_views(d)
        A = interp_matrix(b, -db, n + db, -eb // NREF, (n + eb) // NREF)
        for P in _plane_iter(-db, n + db, n):
            planes = np.take(Phi, P - Phi_lo, axis=d + 1)            # (K, a0, a1) over the table box
            fine = planes[:, eb - db:eb + n + db + 1, eb - db:eb + n + db + 1]
            coarse = planes[:, ::NREF, ::NREF]
            out[(d, P)] = fine - A @ coarse @ A.T
    return out


def _accumulate_annulus(accum, c, tabs, lo, prm):
    """accum[g] += sum_p c_p D_p[g - lo] for the skeleton nodes g of
    Omega_{i,beta} minus Omega_{i,alpha} inside [0, N]^3 (tabs from
    _annulus_plane_tables)."""
    N, n, da, db = prm.N, prm.n, prm.d_alpha, prm.d_beta
    b_lo = np.maximum(lo - db, 0)
    b_hi = np.minimum(lo + n + db, N)
    for d in range(3):
        a0, a1 = _plane_views(d)
        x0 = np.arange(b_lo[a0], b_hi[a0] + 1)
        x1 = np.arange(b_lo[a1], b_hi[a1] + 1)
        keep = _canonical_keep(x0, x1, d, a0, a1, n, (len(x0), len(x1)))
        for P in _plane_iter(b_lo[d], b_hi[d], n):
            in_a_d = (lo[d] - da) <= P <= (lo[d] + n + da)
            inner = (((x0 >= lo[a0] - da) & (x0 <= lo[a0] + n + da))[:, None]
                     & ((x1 >= lo[a1] - da) & (x1 <= lo[a1] + n + da))[None, :])
            mask = keep & ~(inner & in_a_d)
            tab = tabs[(d, P - lo[d])]
            r0 = x0 - lo[a0] + db
            r1 = x1 - lo[a1] + db
            val = np.einsum("k,kxy->xy", c, tab[:, r0[0]:r0[-1] + 1, r1[0]:r1[-1] + 1])
            idx = [None, None, None]
            idx[d] = P
            idx[a0] = slice(x0[0], x0[-1] + 1)
            idx[a1] = slice(x1[0], x1[-1] + 1)
            view = accum[tuple(idx)]
            view += np.where(mask, val, 0.0)


def _interp_coarse_everywhere(phiH, O_lo, prm):
    """I(phi^H)(g) for every skeleton node g (on its canonical plane)."""
    N, n, b = prm.N, prm.n, prm.bb
    out = np.zeros((N + 1,) * 3)
    O_hi = O_lo + phiH.shape[0] - 1
    A = interp_matrix(b, 0, N, O_lo, O_hi)
    xs = np.arange(N + 1)
    for d in range(3):
        a0, a1 = _plane_views(d)
        keep = _canonical_keep(xs, xs, d, a0, a1, n, (N + 1, N + 1))
        for P in range(0, N + 1, n):
            coarse = np.take(phiH, P // NREF - O_lo, axis=d)
            val = A @ coarse @ A.T
            idx = [slice(None)] * 3
            idx[d] = P
            view = out[tuple(idx)]
            view[keep] = val[keep]
    return out


def _boundary_literal(fields, moments, patches, Phi, Phi_lo, phiH, O_lo, prm):
    """phi^B[g] = loc_g(g) + I(phi^H - loc_g)(g) evaluated node by node,
    with loc_g from sec. 4.1 eq. philocmlcII (small problems only)."""
    N, n, b, da, db, e = prm.N, prm.n, prm.bb, prm.d_alpha, prm.d_beta, prm.e
    out = np.zeros((N + 1,) * 3)
    plo = n * patches
    for g in np.argwhere(skeleton_mask(N, n)):
        in_a = np.all((g >= plo - da) & (g <= plo + n + da), axis=1)
        in_b = np.all((g >= plo - db) & (g <= plo + n + db), axis=1) & ~in_a
        Sa = np.nonzero(in_a)[0]
        Sb = np.nonzero(in_b)[0] if Phi is not None else np.zeros(0, dtype=np.int64)

        def loc(y):
            s = 0.0
            for k in Sa:
                r = y - (plo[k] - e)
                s += fields[tuple(patches[k])][tuple(r)]
            for k in Sb:
                r = y - plo[k] - Phi_lo
                s += float(moments[k] @ Phi[(slice(None),) + tuple(r)])
            return s

        d = normal_axis(g, n)
        pts, W = stencil(g, n, b, d)
        val = loc(g)
        for k in range(W.shape[0]):
            for l in range(W.shape[1]):
                if W[k, l] != 0.0:
                    c = pts[k, l]
                    val += W[k, l] * (phiH[tuple(c - O_lo)] - loc(NREF * c))
        out[tuple(g)] = val
    return out


def level_box_margin(prm, deeper=False):
    """Cells of the next coarser level by which its patch box extends past the
    coarsened domain [0, N/Nref] on each side: whole patches, enough that the
    coarse charge (supported on the coarsened Omega_beta regions, margin
    d_beta/Nref) vanishes on the box's outer nodes and its grown region
    (G(C(Omega_beta), b), the interpolation stencils) lies inside it -- the
    proper nesting condition of sec. 5.  When that level has a coarser level
    of its own (deeper), its box must be Nref-aligned in patches as well."""
    need = prm.d_beta // NREF + prm.bb + 1
    m = -(-need // prm.n) * prm.n
    if deeper:
        while ((prm.N // NREF + 2 * m) // NREF) % prm.n or (prm.N // NREF + 2 * m) % NREF:
            m += prm.n
    return m


def mlc_solve_multilevel(f, prm, levels, G1=None, level_alpha=(), rhs_order=4, moments_fn=None):
    """Multilevel MLC (sec. 5) with `levels` levels (2 = the two-level method):
    the two-level steps at the finest level, with the coarse convolution
    replaced by the same method applied one level up to the coarse charge F^H
    (spacing Nref h, the same n, beta, P, Q, b), placed in a patch box that
    extends level_box_margin(prm) cells past the coarsened domain; the
    coarsest level is a single convolution.  The inner radius of the level k
    levels above the finest is level_alpha[k-1] when given and nonzero, else
    that of the next finer level (sec. 7.2 raises alpha at the coarser levels
    to bound the error of the truncated Legendre expansions there).
    rhs_order=6 solves the sixth-order right-hand side of the 27-point
    operator at the finest level instead (see mlc_solve_sixth): the coarser
    levels are unchanged.  moments_fn, if given, supplies the finest level's
    Legendre coefficients as in mlc_solve (the coarser levels take theirs
    from their node charges by Boole's rule).  Every level takes its boundary
    values from the uncorrected discrete solution (phi-tilde) of the level
    below it (sec. 5 eq. mlcmultilevel); the Mehrstellen correction is added
    at the finest level.  Returns phi and, from the finest level down, the
    per-level results (phi-tilde on the level's nodes, or phi^H of the final
    convolution on its output box; the physical coordinate of the array's
    first node; the level's spacing; the level's node charge f-tilde, None
    for the final convolution)."""
    from .dgf import dgf_cached
    if G1 is None:
        G1 = dgf_cached(prm.Q, prm.Z)
    if levels < 2:
        raise ValueError("levels must be >= 2")
    trail = {}

    def solve(fl, p, lv, depth, x0):
        # lv: levels left (2 = this level's coarse solve is a convolution)
        sixth = depth == 0 and rhs_order == 6
        if sixth:
            from .stencils import sixth_order_rhs
            if p.Q != 6:
                raise ValueError("the sixth-order right-hand side is that of the 27-point operator (Q = 6)")
            fl = sixth_order_rhs(fl)
        mfn = moments_fn if depth == 0 else None
        if lv == 2:
            phi, out = mlc_solve(fl, p, G1, keep=True, correct=not sixth, moments_fn=mfn)
            trail[depth + 1] = (out["phiH"], x0 + out["O_lo"] * p.H, p.H, None)
        else:
            m = level_box_margin(p, deeper=lv > 3)
            N1 = p.N // NREF + 2 * m
            a1 = level_alpha[depth] if depth < len(level_alpha) and level_alpha[depth] else p.alpha
            p1 = Params(N=N1, n=p.n, alpha=a1, beta=p.beta, P=p.P, Q=p.Q, b=p.b, h=NREF * p.hh, Z=p.Z)

            def coarse(FH, S_lo, O_lo, O_hi):
                f1 = np.zeros((N1 + 1,) * 3)
                a = S_lo + m                                  # F^H's first node in the level box
                f1[tuple(slice(a, a + FH.shape[d]) for d in range(3))] = FH
                _, out1 = solve(f1, p1, lv - 1, depth + 1, x0 - m * p1.hh)
                o, w = O_lo + m, O_hi - O_lo + 1
                return out1["phitilde"][o:o + w, o:o + w, o:o + w].copy()

            phi, out = mlc_solve(fl, p, G1, keep=True, coarse_fn=coarse, correct=not sixth, moments_fn=mfn)
        trail[depth] = (out["phitilde"], x0, p.hh, fl)
        return phi, out

    phi, _ = solve(f, prm, levels, 0, 0.0)
    return phi, [trail[k] for k in sorted(trail)]


def mlc_solve_sixth(f, prm, G1=None, **kw):
    """Sixth-order variant for the 27-point operator (sec. 2 eq. msCorr; the
    paper specialises its algorithm to fourth order for the simple final
    correction and notes the higher-order form): the method applied to the
    modified right-hand side f~ = stencils.sixth_order_rhs(f), with no final
    correction.  f must vanish within two nodes of the domain's faces."""
    from .stencils import sixth_order_rhs
    if prm.Q != 6:
        raise ValueError("the sixth-order right-hand side is that of the 27-point operator (Q = 6)")
    return mlc_solve(sixth_order_rhs(f), prm, G1, correct=False, **kw)
