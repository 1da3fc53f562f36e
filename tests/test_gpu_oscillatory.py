"""The oscillatory three-charge workload of paper sec. 7.2 (gamma = 28 pi,
Ro = 1/20, the printed centres and closed-form potential) through the
two-level solve with the 27-point operator (MI355X only).

The paper runs this charge with three and four levels at N >= 2048; with two
levels the coarse torus of the DGF table (Z = 128) bounds this build at
N = 416 for 32^3-cell patches.  Checked: element-by-element parity with the
oracle at 128^3 (16^3-cell patches) and 256^3 (32^3-cell patches), float64
1e-12 and float32 2e-6 on phi; at 384^3 the float32 path within 2e-6 of the
float64 one, the patch solves satisfying the Mehrstellen equation, and the
error against the closed form falling as the charge is resolved."""
import os

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from oracle.stencils import apply_laplacian
from paper_1702_08111_amd import mlc as gm

from gpu_common import gpu_solve, oracle_params, rel

pytestmark = pytest.mark.gpu

Q = 6


@pytest.fixture(scope="module")
def closed_form_errors():
    return {}


@pytest.mark.parametrize("N,n", [(128, 16), (256, 32)])
def test_oscillatory_parity(N, n, closed_form_errors):
    f = mi.oscillatory_charge(N)
    exact = mi.oscillatory_potential(N)
    g64 = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp64"), f, keep=False)
    g32 = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp32"), f, keep=False)
    prm = oracle_params(g64["info"], 3.0, 6.0)
    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        o = omlc.mlc_solve(f, prm, dgf_cached(Q, prm.Z))
    e64, e32 = rel(g64["phi"], o), rel(g32["phi"], o)
    ex = float(np.abs(g64["phi"] - exact).max() / np.abs(exact).max())
    closed_form_errors[N] = ex
    print(N, n, f"fp64 vs oracle {e64:.2e}, fp32 vs oracle {e32:.2e}, fp64 vs closed form {ex:.3e}", flush=True)
    assert e64 < 1e-12
    assert e32 < 2e-6


def test_oscillatory_384(closed_form_errors):
    N, n = 384, 32
    f = mi.oscillatory_charge(N)
    exact = mi.oscillatory_potential(N)
    g64 = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp64"), f, keep=True)
    g32 = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp32"), f, keep=False)
    assert g64["info"]["M_coarse"] == 240
    e = rel(g32["phi"], g64["phi"])
    ex = float(np.abs(g64["phi"] - exact).max() / np.abs(exact).max())
    closed_form_errors[N] = ex
    print(N, n, f"fp32 vs fp64 {e:.2e}, fp64 vs closed form {ex:.3e}", flush=True)
    assert e < 2e-6
    # patch solves: Delta^h (phi - h^2 f / 12) = f inside every patch, phi^B on the skeleton
    h = 1.0 / N
    u = g64["phi"] - h * h / 12.0 * f
    inner = ~omlc.skeleton_mask(N, n)[1:-1, 1:-1, 1:-1]
    lap = apply_laplacian(u, Q, h)
    assert rel(lap[inner], f[1:-1, 1:-1, 1:-1][inner]) < 1e-9
    sk = omlc.skeleton_mask(N, n)
    assert np.abs(u[sk] - g64["phiB"][sk]).max() < 1e-14 * np.abs(u).max()
    # the charge is resolved better at every refinement (Ro = 1/20 spans
    # 6.4, 12.8 and 19.2 cells at N = 128, 256, 384)
    if {128, 256} <= set(closed_form_errors):
        errs = [closed_form_errors[k] for k in (128, 256, 384)]
        print("closed-form errors", errs, flush=True)
        assert errs[0] > errs[1] > errs[2]
