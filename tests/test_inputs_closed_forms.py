"""Pins of the closed-form potentials the workloads are checked against
(mlc_inputs): each must solve the radial Poisson equation of its charge,
join its exterior monopole smoothly, and carry the charge's total mass
(the oscillatory charges of sec. 7.2, the compact bumps, the smooth charge
of sec. 7.1)."""
import numpy as np
import pytest
from scipy.integrate import quad

import mlc_inputs as mi


def _radial_laplacian(psi, r, d=2e-4):
    """psi'' + 2 psi' / r by fourth-order central differences."""
    p = [psi(r + k * d) for k in (-2, -1, 0, 1, 2)]
    d2 = (-p[0] + 16 * p[1] - 30 * p[2] + 16 * p[3] - p[4]) / (12 * d * d)
    d1 = (p[0] - 8 * p[1] + 8 * p[3] - p[4]) / (12 * d)
    return d2 + 2 * d1 / r


CASES = {
    # (dimensionless potential psi(r), charge profile rho(r)): Delta psi = rho
    "oscillatory": (lambda r: mi._osc_psi(r), lambda r: mi._osc_profile(r)),
    "bump": (lambda r: mi._psi_bump(r), lambda r: np.where(r < 1, (1 - r * r) ** 4, 0.0)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_closed_form_solves_radial_poisson(name):
    psi, rho = CASES[name]
    r = np.linspace(0.02, 0.98, 97)
    lap = _radial_laplacian(psi, r)
    assert np.abs(lap - rho(r)).max() < 1e-6 * max(np.abs(rho(r)).max(), 1e-3)
    # the exterior is harmonic
    r = np.linspace(1.05, 3.0, 20)
    assert np.abs(_radial_laplacian(psi, r)).max() < 1e-8


@pytest.mark.parametrize("name", sorted(CASES))
def test_closed_form_monopole_and_joins(name):
    psi, rho = CASES[name]
    # exterior psi = -q / r with q = int_0^1 rho r^2 dr (Gauss's law, Delta psi = rho)
    q, _ = quad(lambda r: float(rho(np.array(r))) * r * r, 0, 1, limit=400, epsabs=1e-14)
    for r in (1.5, 2.0, 7.0):
        assert abs(psi(np.array(r)) * r + q) < 1e-12
    # value and slope continuous across r = 1
    e = 1e-7
    v_in = 2 * psi(np.array(1 - e)) - psi(np.array(1 - 2 * e))     # linear extrapolation to r = 1
    v_out = 2 * psi(np.array(1 + e)) - psi(np.array(1 + 2 * e))
    assert abs(v_in - v_out) < 1e-12
    s_in = (psi(np.array(1 - e)) - psi(np.array(1 - 3 * e))) / (2 * e)
    s_out = (psi(np.array(1 + 3 * e)) - psi(np.array(1 + e))) / (2 * e)
    assert abs(s_in - s_out) < 1e-5
    # the centre value is the limit of the interior formula
    assert abs(psi(np.array(0.0)) - psi(np.array(1e-6))) < 1e-9


def test_oscillatory_charge_on_nodes():
    """Three charges of radius 1/20 centred at the printed points; the node
    arrays of charge and potential agree with the profile functions."""
    N = 64
    f = mi.oscillatory_charge(N)
    phi = mi.oscillatory_potential(N)
    assert f.shape == phi.shape == (N + 1,) * 3
    assert np.all(f >= 0) and f[0].max() == 0 and f[-1].max() == 0
    g = np.array([12, 28, 52])          # the node at (3/16, 7/16, 13/16) * 64
    assert f[tuple(g)] == 0.0           # r = 0: (r - r^2)^2 vanishes at the centre
    x = g / N
    want = sum(mi._osc_psi(np.linalg.norm(x - np.array(c)) / mi.OSC_RO) / mi.OSC_RO for c in mi.OSC_CENTRES)
    assert abs(phi[tuple(g)] - want) < 1e-12 * abs(want)
