"""Pins of the two-level MLC oracle as a whole (paper sec. 4.1, sec. 7.1)."""
import numpy as np
import pytest

import mlc_inputs as mi
from oracle import convolution as conv
from oracle import mlc
from oracle.dgf import dgf_cached
from oracle.stencils import apply_laplacian


def _global_discrete(G1, Z, f, N):
    """G^h * f on all nodes, by Hockney over the whole grid, plus the
    Mehrstellen correction h^2 f / 12 (sec. 2 eq. msCorr4)."""
    h = 1.0 / N
    g = conv.conv_hockney(G1, Z, f, np.zeros(3, int), np.full(3, N), M=2 * N + 1)
    return h * h * g


@pytest.mark.parametrize("Q,beta", [(4, 3), (4, 6), (6, 3), (6, 6)])
def test_boundary_values_literal_vs_regrouped(Q, beta):
    """The node-by-node evaluation phi^B = loc_g(g) + I(phi^H - loc_g)(g)
    (sec. 4.1 eqs. philocmlcII, mlcfulldiscr) equals the per-patch
    regrouping used for larger problems (linearity of I)."""
    N, n = 16, 8
    G1 = dgf_cached(Q, 64)
    f = mi.bump_charge(N, [mi.Bump((0.45, 0.5, 0.55), 0.3, 1.0)])
    prm = mlc.Params(N=N, n=n, alpha=3, beta=beta, P=4, Q=Q, Z=64)
    phi1, a = mlc.mlc_solve(f, prm, G1, keep=True)
    phi2, b = mlc.mlc_solve(f, prm, G1, bc_mode="literal", keep=True)
    sk = mlc.skeleton_mask(N, n)
    assert np.abs(a["phiB"] - b["phiB"])[sk].max() < 1e-14 * np.abs(b["phiB"]).max()
    assert np.abs(phi1 - phi2).max() < 1e-14 * np.abs(phi2).max()


@pytest.mark.parametrize("Q", [4, 6])
def test_local_convolution_direct_vs_fft(Q):
    """Both convolution modes of step 1 agree (Hockney is exact)."""
    N, n = 16, 8
    G1 = dgf_cached(Q, 64)
    f = mi.bump_charge(N, [mi.Bump((0.4, 0.55, 0.5), 0.3, 1.0)])
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=Q, Z=64)
    q = mlc.patch_charge(f, n, (1, 0, 1))
    a = mlc.local_field(G1, prm, q, "direct")
    b = mlc.local_field(G1, prm, q, "fft")
    assert np.abs(a - b).max() < 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("Q", [4, 6])
def test_dirichlet_reproduces_discrete_solution(Q):
    """Fed the exact boundary values of the global discrete potential, the
    patch Dirichlet solves (sec. 4.1 eq. last_step_fulldiscr) return it in
    every patch interior (uniqueness of the discrete Dirichlet problem)."""
    N, n = 16, 8
    G1 = dgf_cached(Q, 64)
    f = mi.bump_charge(N, [mi.Bump((0.45, 0.5, 0.52), 0.3, 1.0)])
    u = _global_discrete(G1, 64, f, N)
    for i in mlc.patch_indices(N, n):
        sl = tuple(slice(n * i[d], n * i[d] + n + 1) for d in range(3))
        inner = mlc.dirichlet_solve(u[sl], f[sl], Q, 1.0 / N)
        assert np.abs(inner - u[sl][1:-1, 1:-1, 1:-1]).max() < 1e-14 * np.abs(u).max() * 10


def test_discretisation_is_fourth_order():
    """G^h * f + C2 h^2 f converges to the continuous potential at O(h^4)
    (sec. 2 eq. msCorr4)."""
    G1 = dgf_cached(4, 64)
    bumps = mi.one_bump()
    errs = []
    for N in (16, 32, 64):
        f = mi.bump_charge(N, bumps)
        u = _global_discrete(G1, 64, f, N) + f / (12.0 * N * N)
        ex = mi.bump_potential(N, bumps)
        errs.append(np.abs(u - ex).max() / np.abs(ex).max())
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12, errs


def test_mlc0_barrier_error_falls_with_beta():
    """Barrier error of MLC-0 (beta = alpha) scales like beta^-q: L19,
    doubling beta cuts it by at least ~16 (sec. 7.1, Table 1 discussion)."""
    G1 = dgf_cached(4, 128)
    N, n = 64, 16
    f = mi.smooth_charge(N)
    u = _global_discrete(G1, 128, f, N) + f / (12.0 * N * N)
    errs = []
    for beta in (3, 6):
        prm = mlc.Params(N=N, n=n, alpha=beta, beta=beta, P=4, Q=4, Z=128)
        phi = mlc.mlc_solve(f, prm, G1)
        errs.append(np.abs(phi - u).max() / np.abs(u).max())
    assert errs[0] / errs[1] > 16, errs


def test_legendre_far_field_reduces_error():
    """At fixed alpha, adding the Legendre far field out to beta lowers the
    error, and P = 4 beats P = 1 (Tables 2, 3)."""
    G1 = dgf_cached(4, 128)
    N, n = 64, 16
    f = mi.smooth_charge(N)
    ex = mi.smooth_potential(N)

    def err(alpha, beta, P):
        prm = mlc.Params(N=N, n=n, alpha=alpha, beta=beta, P=P, Q=4, Z=128)
        return np.abs(mlc.mlc_solve(f, prm, G1) - ex).max() / np.abs(ex).max()

    e0 = err(1.5, 1.5, 4)
    e1 = err(1.5, 3, 1)
    e4 = err(1.5, 3, 4)
    assert e4 < e1 < e0, (e0, e1, e4)


def test_linearity():
    N, n = 16, 8
    G1 = dgf_cached(4, 64)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=4, Z=64)
    f1 = mi.bump_charge(N, [mi.Bump((0.4, 0.5, 0.5), 0.3, 1.0)])
    f2 = mi.bump_charge(N, [mi.Bump((0.6, 0.45, 0.55), 0.25, -0.7)])
    a, b = 0.3, -1.7
    lhs = mlc.mlc_solve(a * f1 + b * f2, prm, G1)
    rhs = a * mlc.mlc_solve(f1, prm, G1) + b * mlc.mlc_solve(f2, prm, G1)
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max()


def test_cube_symmetry():
    """A charge invariant under the cube's symmetries gives a potential with
    the same symmetries (the plane choice and the interpolation are
    symmetric)."""
    N, n = 32, 8
    G1 = dgf_cached(6, 64)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=6, Z=64)
    f = mi.bump_charge(N, mi.one_bump())
    phi = mlc.mlc_solve(f, prm, G1)
    s = np.abs(phi).max()
    for perm in [(1, 0, 2), (0, 2, 1), (2, 0, 1)]:
        assert np.abs(phi - np.transpose(phi, perm)).max() < 1e-13 * s
    for ax in range(3):
        assert np.abs(phi - np.flip(phi, ax)).max() < 1e-13 * s


def test_plain_config_error_vs_closed_form():
    """The 32^3 single-bump problem (8^3 patches, alpha=3, beta=6, P=4, L19)
    lands within the O(h^4) discretisation error of the closed form."""
    N, n, Q, bumps = mi.workload("fp64_32")
    G1 = dgf_cached(Q, 64)
    f = mi.bump_charge(N, bumps)
    ex = mi.bump_potential(N, bumps)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=Q, Z=64)
    err = np.abs(mlc.mlc_solve(f, prm, G1) - ex).max() / np.abs(ex).max()
    glob = _global_discrete(G1, 64, f, N) + f / (12.0 * N * N)
    eg = np.abs(glob - ex).max() / np.abs(ex).max()
    assert err < 2 * eg, (err, eg)


def _annulus_pairs(N, n, da, db):
    """(skeleton node, patch) pairs with the node in Omega_beta(i) but not in
    Omega_alpha(i): the pairs whose far field enters phi^B."""
    plo = n * mlc.patch_indices(N, n)
    count = 0
    for g in np.argwhere(mlc.skeleton_mask(N, n)):
        in_a = np.all((g >= plo - da) & (g <= plo + n + da), axis=1)
        in_b = np.all((g >= plo - db) & (g <= plo + n + db), axis=1)
        count += int(np.sum(in_b & ~in_a))
    return count


@pytest.mark.slow
@pytest.mark.parametrize("Q", [4, 6])
def test_boundary_values_literal_vs_regrouped_with_annulus(Q):
    """The same equality as above on a grid wide enough that skeleton nodes
    lie in the annulus Omega_beta(i) minus Omega_alpha(i) of some patches
    (24^3 cells, 8^3-cell patches, alpha = 3, beta = 6), so the regrouped
    far-field terms sum_p c_p [Phi_p - I(Phi_p)] of the large-case path are
    exercised against the node-by-node definition (sec. 4.1 eqs.
    philocmlcII, mlcfulldiscr)."""
    N, n = 24, 8
    G1 = dgf_cached(Q, 64)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=Q, Z=64)
    assert _annulus_pairs(N, n, prm.d_alpha, prm.d_beta) > 1000
    f = mi.bump_charge(N, mi.bumps(3, 41, radius=(0.12, 0.2)))
    phi1, a = mlc.mlc_solve(f, prm, G1, keep=True)
    phi2, b = mlc.mlc_solve(f, prm, G1, bc_mode="literal", keep=True)
    sk = mlc.skeleton_mask(N, n)
    assert np.abs(a["phiB"] - b["phiB"])[sk].max() < 1e-14 * np.abs(b["phiB"]).max()
    assert np.abs(phi1 - phi2).max() < 1e-14 * np.abs(phi2).max()


@pytest.mark.parametrize("Q", [4, 6])
def test_far_field_tables_vs_direct_sum_of_projected_charge(Q):
    """Sum_p c_p Phi_p and sum_p c_p T_p (the tables of the Legendre far
    field, sec. 4.1 step 1, built once per problem class by FFTs, mode by
    mode) equal the literal convolution of the patch's projected charge
    chi_i sum_p c_p Q^p with G^h, and its coarse Mehrstellen Laplacian
    (sec. 2: coarse operators act on samples at the coarse nodes), at sampled
    nodes of the table boxes, including annulus nodes."""
    from oracle import legendre as leg
    from oracle.stencils import apply_laplacian
    N, n, P = 32, 8, 4
    G1 = dgf_cached(Q, 64)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=P, Q=Q, Z=64)
    h, H, R = prm.hh, prm.H, prm.R
    f = mi.bump_charge(N, mi.bumps(2, 43, radius=(0.15, 0.3)))
    i = np.array([1, 2, 1])
    lo = n * i
    c = leg.moments(f[lo[0]:lo[0] + n + 1, lo[1]:lo[1] + n + 1, lo[2]:lo[2] + n + 1], n, P, R)
    # chi_0 times the projected charge, on the nodes of the patch at the origin
    q = mlc.patch_charge(leg.projected_charge(c, n, P, R), n, (0, 0, 0))
    Phi, T, Phi_lo, T_lo = mlc.far_field_tables(G1, prm)
    eb = prm.d_beta + 4 * prm.bb
    rng = np.random.default_rng(7)
    pts = rng.integers(-eb, n + eb + 1, size=(60, 3))
    pts[:3] = [[-eb, -eb, -eb], [n + eb, 0, n // 2], [-prm.d_beta, n + prm.d_alpha + 4, 3]]
    direct = h * h * conv.conv_direct_at(G1, prm.Z, q, pts)
    table = np.array([c @ Phi[(slice(None),) + tuple(x - Phi_lo)] for x in pts])
    assert np.abs(direct - table).max() < 1e-13 * np.abs(direct).max()
    # T at sampled coarse nodes of C(Omega_beta(0)), from 3^3 direct samples
    cb_lo, cb_hi = -prm.d_beta // 4, (n + prm.d_beta) // 4
    cs = rng.integers(cb_lo, cb_hi + 1, size=(12, 3))
    cs[0] = [cb_lo, cb_lo, cb_hi]
    for cc in cs:
        off = np.stack(np.meshgrid(*[np.arange(-1, 2)] * 3, indexing="ij"), -1).reshape(-1, 3)
        samp = h * h * conv.conv_direct_at(G1, prm.Z, q, 4 * (cc + off)).reshape(3, 3, 3)
        lap = apply_laplacian(samp, Q, H)[0, 0, 0]
        tab = c @ T[(slice(None),) + tuple(cc - T_lo)]
        assert abs(lap - tab) < 1e-11 * np.abs(T).max() * np.abs(c).max(), (cc, lap, tab)


def test_multilevel_two_levels_is_the_two_level_method():
    """mlc_solve_multilevel with two levels is mlc_solve (sec. 5 with
    l_max = 1 is the algorithm of sec. 4.1)."""
    N, n = 32, 8
    G1 = dgf_cached(4, 64)
    prm = mlc.Params(N=N, n=n, alpha=3, beta=6, P=4, Q=4, Z=64)
    f = mi.bump_charge(N, mi.one_bump())
    phi, trail = mlc.mlc_solve_multilevel(f, prm, 2, G1)
    assert np.array_equal(phi, mlc.mlc_solve(f, prm, G1))
    assert len(trail) == 2 and trail[1][2] == prm.H


def _three_vs_two(N, n, alpha, beta, Q, Z):
    G1 = dgf_cached(Q, Z)
    f = mi.smooth_charge(N)
    prm = mlc.Params(N=N, n=n, alpha=alpha, beta=beta, P=4, Q=Q, Z=Z)
    p2, o2 = mlc.mlc_solve(f, prm, G1, keep=True)
    p3, trail = mlc.mlc_solve_multilevel(f, prm, 3, G1)
    # the level-1 MLC solution against the exact coarse convolution phi^H it
    # replaces, on phi^H's box
    phiH, O_lo = o2["phiH"], o2["O_lo"]
    m = mlc.level_box_margin(prm)
    o, w = O_lo + m, phiH.shape[0]
    d1 = np.abs(trail[1][0][o:o + w, o:o + w, o:o + w] - phiH).max()
    return f, prm, p2, p3, trail, d1


def test_multilevel_error_propagation_bound():
    """Three levels (sec. 5): the only change from two levels is the coarse
    solution the boundary values interpolate, so the fine-level difference is
    bounded by the level-1 MLC's deviation from the convolution it replaces
    (times the interpolation's and the discrete maximum principle's constants);
    the level box satisfies the proper nesting condition; each level's
    phi-tilde solves its own patch Dirichlet problems."""
    f, prm, p2, p3, trail, d1 = _three_vs_two(64, 8, 3.0, 6.0, 6, 64)
    assert d1 > 1e-12 * np.abs(p2).max()            # the level-1 solve is a real MLC, not exact
    assert np.abs(p3 - p2).max() < 3.0 * d1
    m, N1 = mlc.level_box_margin(prm), trail[1][0].shape[0] - 1
    assert m % prm.n == 0 and N1 == prm.N // 4 + 2 * m
    # F^H (supported on the coarsened Omega_beta regions) vanishes on the box's outer nodes
    fl = trail[1][3]
    assert np.all(fl[0] == 0) and np.all(fl[-1] == 0) and np.all(fl[:, 0] == 0) and np.all(fl[:, :, -1] == 0)
    # level 1: Delta^{h1} phi-tilde = f-tilde at the interior nodes of its patches
    t1, _, h1, _ = trail[1]
    lap = apply_laplacian(t1, prm.Q, h1)
    inner = ~mlc.skeleton_mask(N1, prm.n)[1:-1, 1:-1, 1:-1]
    assert np.abs(lap[inner] - fl[1:-1, 1:-1, 1:-1][inner]).max() < 1e-9 * np.abs(fl).max()


@pytest.mark.slow
def test_multilevel_matches_two_level_when_the_coarse_level_resolves():
    """At 128^3 (16^3-cell patches, L27, alpha 3, beta 6) the level-1 MLC is
    accurate to 2e-6 of phi^H and three levels give the two-level error
    against the closed form within 5 % (sec. 7.1: more levels leave the
    error unchanged when every level is resolved)."""
    f, prm, p2, p3, trail, d1 = _three_vs_two(128, 16, 3.0, 6.0, 6, 128)
    ex = mi.smooth_potential(128)
    e2 = np.abs(p2 - ex).max() / np.abs(ex).max()
    e3 = np.abs(p3 - ex).max() / np.abs(ex).max()
    assert abs(e3 / e2 - 1.0) < 0.05, (e2, e3)


def test_multilevel_coarse_alpha_reduces_level_error():
    """A larger inner radius at the coarser level (sec. 7.2, the remedy for
    the error of the truncated expansions there) leaves that level's charge
    unchanged (F^H depends on the finest level's radii only), reduces the
    level-1 MLC's deviation from the convolution it replaces, and brings the
    fine-level solution to the two-level one (alpha = 2, beta = 3 at the
    finest level; alpha 2 or 3 at level 1: the difference falls by more than
    10, the level-1 deviation over its whole output box by more than 20 %)."""
    N, n, Q, Z = 64, 8, 6, 64
    G1 = dgf_cached(Q, Z)
    f = mi.smooth_charge(N)
    prm = mlc.Params(N=N, n=n, alpha=2.0, beta=3.0, P=4, Q=Q, Z=Z)
    p2, o2 = mlc.mlc_solve(f, prm, G1, keep=True)
    phiH, O_lo = o2["phiH"], o2["O_lo"]
    m = mlc.level_box_margin(prm)
    o, w = O_lo + m, phiH.shape[0]
    res = {}
    for la in ((), (3.0,)):
        p3, trail = mlc.mlc_solve_multilevel(f, prm, 3, G1, level_alpha=la)
        d1 = np.abs(trail[1][0][o:o + w, o:o + w, o:o + w] - phiH).max()
        res[la] = (p3, trail[1][3], d1, np.abs(p3 - p2).max())
    same, wide = res[()], res[(3.0,)]
    assert np.array_equal(same[1], wide[1])
    assert wide[2] < 0.8 * same[2], (same[2], wide[2])
    assert wide[3] < 0.1 * same[3], (same[3], wide[3])
    # an explicit radius equal to the finest level's is the default
    p3, _ = mlc.mlc_solve_multilevel(f, prm, 3, G1, level_alpha=(2.0,))
    assert np.array_equal(p3, same[0])
