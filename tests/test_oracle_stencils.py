"""Pins of the Mehrstellen stencils (paper sec. 2 and appendix A.1)."""
import numpy as np
import pytest

from oracle.stencils import C2, apply_laplacian, stencil_b, stencil_weights, symbol


def _moment(a, px, py, pz):
    s = np.arange(-1, 2)
    return np.sum(a * (s[:, None, None] ** px) * (s[None, :, None] ** py) * (s[None, None, :] ** pz))


@pytest.mark.parametrize("Q", [4, 6])
def test_consistency_identities(Q):
    """Taylor expansion of sum_s a_s u(x + s h) / h^2: consistency with the
    Laplacian needs sum a = 0, sum a s_x^2 = 2, and the truncation error
    C2 h^2 Delta^2 u with C2 = 1/12 (sec. 2) needs sum a s_x^4 = 24 C2 = 2
    and sum a s_x^2 s_y^2 = 8 C2 = 2/3."""
    a = stencil_weights(Q)
    assert abs(_moment(a, 0, 0, 0)) < 1e-14
    for p in [(2, 0, 0), (0, 2, 0), (0, 0, 2)]:
        assert abs(_moment(a, *p) - 2.0) < 1e-14
    for p in [(4, 0, 0), (0, 4, 0), (0, 0, 4)]:
        assert abs(_moment(a, *p) - 24 * C2) < 1e-14
    for p in [(2, 2, 0), (0, 2, 2), (2, 0, 2)]:
        assert abs(_moment(a, *p) - 8 * C2) < 1e-14
    # odd moments vanish by symmetry
    assert abs(_moment(a, 1, 0, 0)) < 1e-14 and abs(_moment(a, 1, 1, 1)) < 1e-14


def test_l27_sixth_order_moments():
    """The L27 truncation error in appendix A.1 has the h^4 term
    (1/360)(Delta^2 + 2 (dxxyy + dyyzz + dzzxx)) Delta u.  For a homogeneous
    sixth-degree monomial u the h = 1 stencil applied at the origin is
    exactly sum_s a_s u(s) (only the sixth Taylor term survives), and the
    right side reduces to that h^4 term, so the two must agree monomial by
    monomial."""
    a = stencil_weights(6)
    import itertools
    import math

    def stencil_on_monomial(px, py, pz):
        return _moment(a, px, py, pz)

    def paper_h4_term(px, py, pz):
        # (1/360) (Delta^2 + 2 (d^4/dx^2dy^2 + ...)) Delta u at 0 for u = x^px y^py z^pz,
        # i.e. (1/360) * sum over sixth-derivative multi-indices with the weights
        # of the operator (Delta^3 + 2 Delta (mixed quartic)).
        ops = {}
        # Delta^3 = sum over (i,j,k) of dx^2i dy^2j dz^2k with multinomial 3!/(i!j!k!)
        for i, j, k in itertools.product(range(4), repeat=3):
            if i + j + k == 3:
                ops[(2 * i, 2 * j, 2 * k)] = ops.get((2 * i, 2 * j, 2 * k), 0) + \
                    math.factorial(3) // (math.factorial(i) * math.factorial(j) * math.factorial(k))
        mixed = [(2, 2, 0), (0, 2, 2), (2, 0, 2)]
        for m in mixed:
            for d in [(2, 0, 0), (0, 2, 0), (0, 0, 2)]:
                key = tuple(x + y for x, y in zip(m, d))
                ops[key] = ops.get(key, 0) + 2
        c = ops.get((px, py, pz), 0)
        return c * math.factorial(px) * math.factorial(py) * math.factorial(pz) / 360.0

    for px, py, pz in itertools.product(range(7), repeat=3):
        if px + py + pz != 6:
            continue
        # stencil applied to the monomial at the origin (h = 1)
        lhs = stencil_on_monomial(px, py, pz)
        # (s.grad)^6 u / 6! at 0 reproduces the monomial itself, so the
        # stencil value is the h^4 truncation coefficient of that monomial
        assert abs(lhs - paper_h4_term(px, py, pz)) < 1e-13, (px, py, pz)


@pytest.mark.parametrize("Q,slope", [(4, -7.0), (6, -9.0)])
def test_figure1_truncation_slopes(Q, slope):
    """Fig. 1: log10 |Delta^{h=1} S(G)| against log10 |g|_inf has slope -7
    (L19) and -9 (L27) away from the singularity."""
    L = 34
    ax = np.arange(-L, L + 1, dtype=np.float64)
    r = np.sqrt(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
    r[L, L, L] = 1.0
    G = -1.0 / (4 * np.pi * r)
    tau = apply_laplacian(G, Q)
    g = np.arange(-L + 1, L)
    rinf = np.maximum(np.maximum(np.abs(g)[:, None, None], np.abs(g)[None, :, None]), np.abs(g)[None, None, :])
    rs = np.arange(6, 25)
    env = np.array([np.abs(tau[rinf == k]).max() for k in rs])
    fit = np.polyfit(np.log10(rs), np.log10(env), 1)[0]
    assert abs(fit - slope) < 0.25, fit


@pytest.mark.parametrize("Q", [2, 4, 6])
def test_symbol_matches_stencil(Q):
    """The DST eigenvalue formula equals the stencil applied to a sine mode."""
    n = 12
    m = np.arange(1, n)
    k = (3, 5, 8)
    mode = (np.sin(np.pi * k[0] * np.arange(0, n + 1) / n)[:, None, None]
            * np.sin(np.pi * k[1] * np.arange(0, n + 1) / n)[None, :, None]
            * np.sin(np.pi * k[2] * np.arange(0, n + 1) / n)[None, None, :])
    lap = apply_laplacian(mode, Q)
    c = [np.cos(np.pi * kk / n) for kk in k]
    lam = symbol(Q, *c)
    assert np.allclose(lap, lam * mode[1:-1, 1:-1, 1:-1], atol=1e-13)
    assert len(m) == n - 1


def test_stencil_coefficients_from_paper():
    """The oracle's weights equal the appendix's printed values
    (tests/golden/mehrstellen_coefficients.txt)."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "mehrstellen_coefficients.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 2
    for Q, *bs in rows:
        want = [float(Fraction(b)) for b in bs]
        assert stencil_b(int(Q)) == pytest.approx(want, abs=1e-16), Q
