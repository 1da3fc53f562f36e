"""Pins of the sixth-order variant for the 27-point operator (sec. 2 eq.
msCorr with the h^4 term of that operator's truncation error, appendix A.1):
the modified right-hand side f~ is built from differences of f, and the
discrete solution G^h * f~ needs no final correction."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

import mlc_inputs as mi
from oracle import convolution as conv
from oracle import mlc
from oracle.stencils import C2, apply_laplacian, sixth_order_rhs, sixth_order_rhs_stencil


def _poly3(c, x, y, z):
    return npoly.polyval3d(x, y, z, c)


def _deriv(c, ax, m):
    return npoly.polyder(c, m=m, axis=ax) if m else c


def test_closed_form_potential_of_the_polynomial_charge():
    """mlc_inputs.poly_potential solves Delta phi = poly_charge: the 7-point
    Laplacian of its samples approaches the charge at second order."""
    res = []
    for N in (32, 64):
        phi, f = mi.poly_potential(N), mi.poly_charge(N)
        h = 1.0 / N
        lap = (phi[2:, 1:-1, 1:-1] + phi[:-2, 1:-1, 1:-1] + phi[1:-1, 2:, 1:-1] + phi[1:-1, :-2, 1:-1]
               + phi[1:-1, 1:-1, 2:] + phi[1:-1, 1:-1, :-2] - 6.0 * phi[1:-1, 1:-1, 1:-1]) / (h * h)
        res.append(np.abs(lap - f[1:-1, 1:-1, 1:-1]).max())
    assert 3.6 < res[0] / res[1] < 4.4, res
    # and the potential decays like -Q / (4 pi r) with Q the total charge
    k, R = 10, 0.3
    m2, _ = mi._poly_profile_integrals(k)
    Q = 4.0 * np.pi * R ** 3 * npoly.polyval(1.0, m2)
    phi = mi.poly_potential(64, k, (0.5, 0.5, 0.5), R)
    assert abs(phi[0, 32, 32] - (-Q / (4.0 * np.pi * 0.5))) < 1e-14


def test_rhs_is_the_continuous_correction_on_quintics():
    """On polynomials of total degree <= 5 every difference in f~ is exact, so
    f~ = f + (h^2/12) Delta f + (h^4/360) (sum_d d_d^4 + 4 sum_{d<e} d_d^2 d_e^2) f
    with the derivatives taken exactly (the h^4 operator is the appendix's
    Delta^2 + 2 (d_xxyy + d_yyzz + d_zzxx))."""
    rng = np.random.default_rng(7)
    c = np.zeros((6, 6, 6))
    for i in range(6):
        for j in range(6 - i):
            for k in range(6 - i - j):
                c[i, j, k] = rng.standard_normal()
    h = 0.05
    g = np.arange(-6, 7) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    f = _poly3(c, X, Y, Z)
    got = sixth_order_rhs_stencil(f)[2:-2, 2:-2, 2:-2]
    sl = (slice(2, -2),) * 3
    lap = sum(_poly3(_deriv(c, d, 2), X, Y, Z) for d in range(3))
    quart = sum(_poly3(_deriv(c, d, 4), X, Y, Z) for d in range(3))
    mixed = sum(_poly3(_deriv(_deriv(c, d, 2), e, 2), X, Y, Z) for d in range(3) for e in range(d + 1, 3))
    want = f + h * h * C2 * lap + h ** 4 / 360.0 * (quart + 4.0 * mixed)
    assert np.abs(got - want[sl]).max() < 1e-12 * np.abs(want).max()
    # the same operator written as Delta^2 + 2 sum d_xxyy
    bih = sum(_poly3(_deriv(_deriv(c, d, 2), e, 2), X, Y, Z) for d in range(3) for e in range(3))
    assert np.allclose(quart + 4.0 * mixed, bih + 2.0 * mixed, atol=1e-9)


def test_truncation_is_sixth_order():
    """The 27-point operator applied to the exact potential's samples equals
    f~ up to O(h^6) (and f + C2 h^2 Delta_h f only up to O(h^4))."""
    r6, r4 = [], []
    for N in (32, 64):
        phi, f = mi.poly_potential(N), mi.poly_charge(N)
        h = 1.0 / N
        L = apply_laplacian(phi, 6, h)
        r6.append(np.abs(L - sixth_order_rhs(f)[1:-1, 1:-1, 1:-1]).max())
        r4.append(np.abs(L - (f[1:-1, 1:-1, 1:-1] + C2 * apply_laplacian(f, 6, 1.0))).max())
    assert r6[0] / r6[1] > 50, r6
    assert 12 < r4[0] / r4[1] < 20, r4


def test_discrete_solution_is_sixth_order(dgf64_q6):
    """G^h * f~ approaches the closed-form potential at sixth order (ratio 64
    per halving of h), where G^h * f + C2 h^2 f does at fourth (16)."""
    e6, e4 = [], []
    for N in (32, 64):
        f, ex = mi.poly_charge(N), mi.poly_potential(N)
        h = 1.0 / N
        lo, hi = np.zeros(3, int), np.full(3, N)
        d6 = conv.conv_hockney(dgf64_q6, 64, sixth_order_rhs(f), lo, hi, M=2 * N + 1) * h * h
        d4 = conv.conv_hockney(dgf64_q6, 64, f, lo, hi, M=2 * N + 1) * h * h + C2 * h * h * f
        e6.append(np.abs(d6 - ex).max() / np.abs(ex).max())
        e4.append(np.abs(d4 - ex).max() / np.abs(ex).max())
    assert e6[0] / e6[1] > 45, e6
    assert 13 < e4[0] / e4[1] < 19, e4
    assert e6[1] < e4[1] / 50


def test_sixth_order_preconditions():
    f = mi.poly_charge(32)
    with pytest.raises(ValueError):
        mlc.mlc_solve_sixth(f, mlc.Params(N=32, n=8, alpha=3, beta=6, P=4, Q=4, Z=64))
    bad = f.copy()
    bad[2, 16, 16] = 1.0        # inside the two-node band along the faces
    with pytest.raises(ValueError):
        sixth_order_rhs(bad)
    ft = sixth_order_rhs(f)
    assert abs(ft.sum() - f.sum()) < 1e-12 * abs(f.sum())   # the differences carry no net charge
