"""Pins of the oracle's Gauss-integrated Legendre coefficients for charges
given analytically (paper sec. 4.1 step 1; sec. 3 projection)."""
import numpy as np
import pytest

import mlc_inputs as mi
from oracle import legendre as leg


def _poly_charge(c, P, corner, R):
    """sum_p c_p Q^p on the patch with low corner `corner` and half-width R."""
    def fun(x0, x1, x2):
        t = [(x0 - corner[0]) / R - 1.0, (x1 - corner[1]) / R - 1.0, (x2 - corner[2]) / R - 1.0]
        return sum(ck * R ** -1.5 * leg.qhat(p[0], t[0]) * leg.qhat(p[1], t[1]) * leg.qhat(p[2], t[2])
                   for ck, p in zip(c, leg.mode_list(P)))
    return fun


@pytest.mark.parametrize("P,g", [(1, 1), (2, 2), (3, 3), (4, 4), (5, 5), (6, 6)])
def test_gauss_reproduces_polynomials(P, g):
    """With 2g - 1 >= 2(P - 1) the composite rule integrates every product of
    two modes exactly, so the coefficients of a charge of degree < P come back
    exactly (the rule's value of <Q^p, f> is the exact inner product)."""
    n, h = 8, 1.0 / 32
    R = n * h / 2
    corner = np.array([0.25, 0.5, 0.25])
    c = np.random.default_rng(P).standard_normal(len(leg.mode_list(P)))
    got = leg.moments_gauss(_poly_charge(c, P, corner, R), corner, n, h, P, R, g)
    assert np.abs(got - c).max() < 1e-13 * max(1.0, np.abs(c).max())


def test_gauss_rule_too_coarse_is_not_exact():
    """The same with one point too few per cell leaves an error (the pin above
    is sensitive to the rule's degree)."""
    n, h, P = 8, 1.0 / 32, 4
    R = n * h / 2
    corner = np.array([0.25, 0.5, 0.25])
    c = np.random.default_rng(4).standard_normal(len(leg.mode_list(P)))
    got = leg.moments_gauss(_poly_charge(c, P, corner, R), corner, n, h, P, R, 3)
    assert np.abs(got - c).max() > 1e-8


def test_gauss_and_boole_agree_at_sixth_order():
    """For a smooth charge the Gauss coefficients and the Boole ones from node
    values (with the Gram correction) converge together like h^6 when the
    same physical patch is resolved by n = 8, 16, 32 cells."""
    terms = [((0.31, 0.27, 0.36), 0.6, 1.0, 0.0, mi.PROFILE_BUMP)]   # smooth over the whole patch
    corner, side, P = np.array([0.25, 0.25, 0.25]), 0.125, 4
    R = side / 2
    diffs = []
    for n in (8, 16, 32):
        h = side / n
        ax = [corner[d] + h * np.arange(n + 1) for d in range(3)]
        fnodes = mi.radial_charge_at(ax[0][:, None, None], ax[1][None, :, None], ax[2][None, None, :], terms)
        cb = leg.moments(fnodes, n, P, R)
        cg = leg.moments_gauss(lambda a, b, c: mi.radial_charge_at(a, b, c, terms), corner, n, h, P, R, 4)
        diffs.append(np.abs(cb - cg).max() / np.abs(cg).max())
    assert diffs[0] / diffs[1] > 30 and diffs[1] / diffs[2] > 30, diffs


def test_radial_terms_match_the_workload_charges():
    """The radial-term forms of the workloads sample to the same node arrays."""
    N = 64
    b = mi.bumps(3, 7)
    assert np.abs(mi.radial_charge_nodes(N, mi.bump_terms(b)) - mi.bump_charge(N, b)).max() < 1e-15
    assert np.abs(mi.radial_charge_nodes(N, mi.smooth_terms()) - mi.smooth_charge(N)).max() < 1e-15
    o = mi.oscillatory_charge(N)
    assert np.abs(mi.radial_charge_nodes(N, mi.oscillatory_terms()) - o).max() < 1e-12 * np.abs(o).max()
