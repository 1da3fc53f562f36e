"""Pins of the local convolution (appendix A.2), the Legendre projection
(sec. 3, sec. 4.1) and the coplanar interpolation (sec. 3.1, 4.1)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import convolution as conv
from oracle import legendre as leg
from oracle.interp import lagrange_weights, stencil
from oracle.mlc import interp_matrix


# ---------------------------------------------------------------- Hockney
@pytest.mark.parametrize("M", [None, 40, 45])
def test_hockney_equals_direct_sum(dgf64_q4, M):
    """Hockney's method computes the free-space discrete convolution exactly
    (appendix A.2): equal to the literal sum up to round-off for any torus
    at least as large as the minimum."""
    rng = np.random.default_rng(1)
    q = rng.standard_normal((7, 9, 8))
    olo, ohi = np.array([-12, -5, -9]), np.array([18, 20, 15])
    d = conv.conv_direct(dgf64_q4, 64, q, olo, ohi)
    hk = conv.conv_hockney(dgf64_q4, 64, q, olo, ohi, M=M)
    assert np.abs(d - hk).max() < 1e-13 * np.abs(d).max()


def test_hockney_rejects_small_torus(dgf64_q4):
    q = np.ones((5, 5, 5))
    with pytest.raises(ValueError):
        conv.conv_hockney(dgf64_q4, 64, q, np.zeros(3, int), np.full(3, 20), M=24)


def test_direct_sum_at_points(dgf64_q4):
    rng = np.random.default_rng(2)
    q = rng.standard_normal((5, 6, 4))
    olo, ohi = np.array([-3, -3, -3]), np.array([8, 8, 8])
    d = conv.conv_direct(dgf64_q4, 64, q, olo, ohi)
    pts = np.array([[0, 0, 0], [8, -3, 2], [-3, 5, 8]])
    v = conv.conv_direct_at(dgf64_q4, 64, q, pts)
    assert np.allclose(v, [d[tuple(p - olo)] for p in pts], rtol=0, atol=1e-15)


# ---------------------------------------------------------------- Legendre
def test_mode_count():
    """K = P(P+1)(P+2)/6: 20 coefficients per patch for P = 4 (abstract, sec. 6)."""
    assert [len(leg.mode_list(P)) for P in (1, 2, 3, 4, 5)] == [1, 4, 10, 20, 35]


def test_boole_panel_is_newton_cotes():
    """One panel of the composite rule is the 5-point closed Newton-Cotes
    (Boole) rule: weights from scipy.integrate.newton_cotes."""
    an, _ = integrate.newton_cotes(4, 1)
    w = leg.boole_weights(4)            # one panel on [-1, 1], step 1/2
    assert np.allclose(w, an * 0.5, atol=1e-15)


@pytest.mark.parametrize("n", [8, 16, 32])
def test_boole_exactness(n):
    """Composite Boole integrates polynomials up to degree 5 exactly and has
    an O(h^6) error at degree 6."""
    t = leg.patch_coords(n)
    w = leg.boole_weights(n)
    for k in range(6):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * t ** k) - exact) < 1e-14
    err6 = abs(np.sum(w * t ** 6) - 2.0 / 7.0)
    assert 0 < err6 < 20 * (2.0 / n) ** 6


def test_orthonormal_basis_by_gauss():
    """Qhat_a are orthonormal on [-1, 1] (Gauss-Legendre, independent of Boole)."""
    x, wg = np.polynomial.legendre.leggauss(12)
    for a in range(9):
        for c in range(9):
            v = np.sum(wg * leg.qhat(a, x) * leg.qhat(c, x))
            assert abs(v - (a == c)) < 1e-14


@pytest.mark.parametrize("P", [1, 2, 4, 5, 6, 9])
def test_projection_reproduces_polynomials(P):
    """P(pi) = pi for polynomials of total degree < P (sec. 3.2 error
    analysis uses this); with the Boole Gram correction this holds exactly."""
    n, R = 16, 0.25
    rng = np.random.default_rng(P)
    c = rng.standard_normal(len(leg.mode_list(P)))
    poly = leg.projected_charge(c, n, P, R)
    c2 = leg.moments(poly, n, P, R)
    assert np.abs(c2 - c).max() < 1e-12
    assert np.abs(leg.projected_charge(c2, n, P, R) - poly).max() < 1e-12 * np.abs(poly).max()


@pytest.mark.parametrize("P", [5, 6, 9])
def test_gram_not_diagonal_above_p4(P):
    """From P = 5 on the Boole rule no longer integrates every product of two
    modes exactly: same-parity pairs of total degree >= 6 couple, so the
    projection needs the full Gram matrix (the moments are not the raw Boole
    moments divided by a diagonal); the coupling vanishes as the patch is
    refined."""
    offs = []
    for n in (8, 16, 32):
        G = leg.gram(n, P)
        off = np.abs(G - np.diag(np.diag(G))).max()
        offs.append(off)
        assert np.abs(G - G.T).max() < 1e-14
    assert offs[0] > 1e-6
    assert offs[0] > offs[1] > offs[2]


def test_gram_diagonal_for_p4():
    """For P <= 4 the Boole Gram matrix is diagonal (Boole is exact to degree
    5, and odd products vanish by symmetry); only the pure cubic modes have a
    diagonal entry different from 1, and it tends to 1 like h^6."""
    for n in (8, 16, 32):
        G = leg.gram(n, 4)
        off = G - np.diag(np.diag(G))
        assert np.abs(off).max() < 1e-14
        d = np.diag(G) - 1.0
        cubic = [k for k, p in enumerate(leg.mode_list(4)) if max(p) == 3]
        assert len(cubic) == 3
        assert np.abs(np.delete(d, cubic)).max() < 1e-14
        assert np.all(d[cubic] > 0) and np.all(d[cubic] < 2 * (2.0 / n) ** 6 * 400)


def test_moments_of_constant_charge():
    """The monomode coefficient of f = 1 on a patch of radius R is
    <Q^0, 1> = R^{-3/2} 2^{-3/2} (2R)^3 = (2R)^{3/2}."""
    n, R = 16, 0.125
    c = leg.moments(np.ones((n + 1,) * 3), n, 4, R)
    assert abs(c[0] - (2 * R) ** 1.5) < 1e-14
    assert np.abs(c[1:]).max() < 1e-15


# ---------------------------------------------------------------- interpolation
@pytest.mark.parametrize("b", [1, 2, 3])
def test_lagrange_exact_to_degree(b):
    nodes = np.arange(-b, b + 2)
    for th in (0.0, 0.25, 0.5, 0.75):
        w = lagrange_weights(b, th)
        for k in range(2 * b + 2):
            assert abs(np.sum(w * nodes ** k) - th ** k) < 1e-13
        if th == 0.0:
            assert np.all(w[nodes != 0] == 0.0) and w[nodes == 0][0] == 1.0


@pytest.mark.parametrize("b", [2, 3])
def test_lagrange_mirror_symmetry(b):
    for th in (0.25, 0.5):
        w = lagrange_weights(b, th)
        wm = lagrange_weights(b, 1 - th)
        assert np.allclose(w, wm[::-1], atol=1e-15)


@pytest.mark.parametrize("b,qi", [(2, 6), (3, 8)])
def test_interpolation_order(b, qi):
    """Interpolating exp-type data from a coarse grid of spacing H converges
    at order q_I = 2b + 2 (sec. 7.1: b=2 gives 6, b=3 gives 8)."""
    errs = []
    for H in (0.2, 0.1, 0.05):
        nf = 64
        A = interp_matrix(b, 16, 16 + nf, 4 - b - 1, 4 + nf // 4 + b + 1)
        xs = np.arange(16, 16 + nf + 1) * H / 4
        cs = np.arange(4 - b - 1, 4 + nf // 4 + b + 2) * H
        errs.append(np.abs(A @ np.sin(3 * cs) - np.sin(3 * xs)).max())
    rate = np.log2(errs[1] / errs[2])
    assert rate > qi - 0.6, (errs, rate)


def test_plane_choice_irrelevant_on_edges():
    """An edge node lies on two face planes; both give the same stencil
    weights on the same coarse nodes (the in-plane axis along the other face
    has theta = 0)."""
    n, b = 8, 2
    g = np.array([16, 8, 13])
    p0, w0 = stencil(g, n, b, 0)
    p1, w1 = stencil(g, n, b, 1)
    vals0 = {tuple(p): w for p, w in zip(p0.reshape(-1, 3), w0.ravel()) if w != 0}
    vals1 = {tuple(p): w for p, w in zip(p1.reshape(-1, 3), w1.ravel()) if w != 0}
    assert vals0.keys() == vals1.keys()
    for k in vals0:
        assert abs(vals0[k] - vals1[k]) < 1e-15
