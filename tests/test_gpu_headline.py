"""Element-by-element parity with the oracle at the benchmark's size
(MI355X only): 256^3 cells, 32^3-cell patches (512), alpha = 3, beta = 6,
P = 4, in both readings of the workload -- the 27-point operator (Q = 6,
local torus M = 160, the benchmark's plan) and the 19-point one (Q = 4,
M = 150) -- with the plans bench.py times.

One full oracle solve per reading (paper sec. 4.1 steps 1-3 and the final
correction, float64, SciPy FFTs on every host core) supplies F^H, phi^H,
phi^B, phi, the moments and, through its local-field hook, the coarse
samples and plane corrections of every patch's local field.  Bars: the
float64 path within 1e-12 relative max-norm on every quantity; the
float32-convolution path within 2e-6 on phi, and within 1e-12 on the
moments (float64 in both paths)."""
import os

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import gpu_solve, local_views, oracle_params, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-6

READINGS = {"q6_m160": ("fp32_256_q6", 160), "q4_m150": ("fp32_256_q4", 150)}


@pytest.fixture(scope="module", params=sorted(READINGS))
def headline(request):
    name, M = READINGS[request.param]
    N, n, Q, bumps = mi.workload(name)
    f = mi.bump_charge(N, bumps)
    gpu = {}
    for conv in ("fp64", "fp32"):
        gpu[conv] = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, fft_size=M), f)
        assert gpu[conv]["info"]["M"] == M
    prm = oracle_params(gpu["fp64"]["info"], 3.0, 6.0)
    info = gpu["fp64"]["info"]
    npch = info["npatch"]
    lc = np.empty((npch, info["Wc"], info["Wc"], info["Wc"]))
    ld = np.empty((npch, 3, info["nplanes_a"], info["Wa"], info["Wa"]))

    def keep_local(pi, i, arr):
        lc[pi], ld[pi] = local_views(prm, arr)

    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        phi, o = omlc.mlc_solve(f, prm, dgf_cached(Q, prm.Z), keep=True, on_local=keep_local)
    o["phi"] = phi
    o["local_coarse"] = lc
    o["local_delta"] = ld
    return request.param, f, gpu, o


def _errors(g, o, N, n):
    sk = omlc.skeleton_mask(N, n)
    return {
        "moments": rel(g["moments"], o["moments"]),
        "FH": rel(g["FH"], o["FH"]),
        "phiH": rel(g["phiH"], o["phiH"]),
        "phiB": rel(g["phiB"][sk], o["phiB"][sk]),
        "phi": rel(g["phi"], o["phi"]),
        "local_coarse": rel(g["local_coarse"], o["local_coarse"]),
        # plane corrections are differences of nearly equal values: their
        # error is measured against the scale of the local fields
        "local_delta": float(np.abs(g["local_delta"] - o["local_delta"]).max() / np.abs(o["local_coarse"]).max()),
    }


def test_fp64_every_quantity(headline):
    tag, f, gpu, o = headline
    info = gpu["fp64"]["info"]
    errs = _errors(gpu["fp64"], o, info["N"], info["n"])
    print(tag, "fp64", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < TOL64, (k, v)


def test_fp32_phi(headline):
    tag, f, gpu, o = headline
    info = gpu["fp32"]["info"]
    errs = _errors(gpu["fp32"], o, info["N"], info["n"])
    print(tag, "fp32", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["phi"] < TOL32, errs
    assert errs["moments"] < TOL64, errs
    assert errs["local_coarse"] < TOL32, errs
