"""Legendre expansion of a patch charge (paper sec. 3, eq. for the
projection P(f^i) and the 3-D Legendre basis; sec. 4.1 step 1 for the
composite quadrature).

Reading used (the paper calls Q^p the classical Legendre polynomial but
writes the projection as sum <Q^p, f> Q^p, which is a projection only for an
orthonormal basis): Q^p(x) = R^{-3/2} prod_d Qhat_{p_d}((x_d - c_d)/R) with
Qhat_a(t) = sqrt((2a+1)/2) P_a(t), orthonormal on [-1, 1].  The discrete
projection is the orthogonal projection in the inner product defined by the
composite Boole rule on the (n+1)^3 patch nodes, applied to f on the closed
patch (the Boole end weights already integrate over [0, nh]).
"""
import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def mode_list(P):
    """Exponent triples p with |p|_1 < P, ordered by total degree, then
    lexicographically descending (p0 first).  len = P(P+1)(P+2)/6."""
    modes = []
    for deg in range(P):
        blk = [p for p in itertools.product(range(deg + 1), repeat=3) if sum(p) == deg]
        modes.extend(sorted(blk, reverse=True))
    return modes


def qhat(a, t):
    """Orthonormal Legendre polynomial sqrt((2a+1)/2) P_a(t)."""
    c = np.zeros(a + 1)
    c[a] = 1.0
    return np.sqrt((2 * a + 1) / 2.0) * npleg.legval(t, c)


def boole_weights(n):
    """Composite Boole weights on [-1, 1] with n panels of width 2/n
    (n % 4 == 0): (2 delta / 45) * [7, 32, 12, 32, 14, 32, ..., 32, 7]."""
    if n % 4:
        raise ValueError("Boole's rule needs n divisible by 4")
    d = 2.0 / n
    w = np.zeros(n + 1)
    for k in range(0, n, 4):
        w[k:k + 5] += np.array([7.0, 32.0, 12.0, 32.0, 7.0])
    return w * (2.0 * d / 45.0)


def patch_coords(n):
    """t_k = (k - n/2) / (n/2), k = 0..n: the patch nodes mapped to [-1, 1]."""
    return (np.arange(n + 1) - n / 2.0) / (n / 2.0)


def gram(n, P):
    """Gram matrix <Qhat_p, Qhat_q> under the tensor Boole rule, for the
    modes of mode_list(P)."""
    t = patch_coords(n)
    w = boole_weights(n)
    m1 = np.array([[np.sum(w * qhat(a, t) * qhat(c, t)) for c in range(P)] for a in range(P)])
    modes = mode_list(P)
    K = len(modes)
    Gm = np.empty((K, K))
    for r, p in enumerate(modes):
        for s, q in enumerate(modes):
            Gm[r, s] = m1[p[0], q[0]] * m1[p[1], q[1]] * m1[p[2], q[2]]
    return Gm


def basis_on_patch(n, P):
    """Qhat_p(t_j) for every mode p and patch node j: shape (K, n+1, n+1, n+1)."""
    t = patch_coords(n)
    vals = [qhat(a, t) for a in range(P)]
    modes = mode_list(P)
    return np.stack([vals[p[0]][:, None, None] * vals[p[1]][None, :, None] * vals[p[2]][None, None, :]
                     for p in modes])


def moments(fpatch, n, P, R):
    """Coefficients c_p of the discrete projection of the patch charge.

    fpatch: f on the (n+1)^3 nodes of the closed patch.  R = n h / 2.
      raw moment  m_p = R^{3/2} sum_j W_j f[j] Qhat_p(t_j)       (Boole)
      projection  c = Gram^{-1} m                                (orthogonal
                  projection in the Boole inner product; for P <= 4 the
                  Gram matrix is diagonal)
    The projected charge is then sum_p c_p Q^p = R^{-3/2} sum_p c_p Qhat_p.
    """
    w = boole_weights(n)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    B = basis_on_patch(n, P)
    m = R ** 1.5 * np.einsum("kabc,abc->k", B, W * fpatch)
    return np.linalg.solve(gram(n, P), m)


def projected_charge(c, n, P, R):
    """sum_p c_p Q^p(x_j) on the patch nodes (no chi weighting)."""
    B = basis_on_patch(n, P)
    return R ** -1.5 * np.einsum("k,kabc->abc", c, B)


def gauss_cell_rule(g):
    """Composite Gauss-Legendre rule on [-1, 1] split into n cells of width
    2/n, g points per cell: returns a function n -> (t, w)."""
    xi, om = np.polynomial.legendre.leggauss(g)

    def rule(n):
        cells = np.arange(n)[:, None]
        t = (cells + 0.5 * (1.0 + xi[None, :])) * (2.0 / n) - 1.0
        w = np.broadcast_to(om[None, :] / n, t.shape)
        return t.reshape(-1), w.reshape(-1)
    return rule


def moments_gauss(fun, corner, n, h, P, R, g):
    """Legendre coefficients of an analytically given charge on the patch
    corner + [0, n h]^3 by composite Gauss integration (sec. 4.1 step 1, for
    f specified analytically): c_p = R^{3/2} sum_k W_k f(x_k) Qhat_p(t_k), the
    Gauss value of the inner product <Q^p, f> of the orthogonal projection
    (sec. 3); g points per cell and axis.  fun(x0, x1, x2) takes arrays that
    broadcast."""
    t, w = gauss_cell_rule(g)(n)
    x = [corner[d] + (t + 1.0) * (n * h / 2.0) for d in range(3)]
    F = fun(x[0][:, None, None], x[1][None, :, None], x[2][None, None, :])
    F = np.asarray(F, dtype=np.float64) * np.ones((len(t),) * 3)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    vals = [qhat(a, t) for a in range(P)]
    out = []
    for p in mode_list(P):
        B = vals[p[0]][:, None, None] * vals[p[1]][None, :, None] * vals[p[2]][None, None, :]
        out.append(R ** 1.5 * np.sum(W * B * F))
    return np.array(out)

