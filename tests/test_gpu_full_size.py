"""GPU checks at the benchmark's full sizes (MI355X only).

128^3 (16^3-cell patches, 96^3 local torus, L19): every output against the
full oracle solve.  256^3 (32^3-cell patches, L27), the benchmark's
workload with the plans bench.py times: invariants that hold at any size
(the coarse solve inverts Delta^H, the patch solves satisfy the Mehrstellen
equation with the final correction); its element-by-element parity with
the oracle is tests/test_gpu_headline.py."""
import numpy as np
import pytest

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from oracle.stencils import apply_laplacian
from paper_1702_08111_amd import mlc as gm

from gpu_common import gpu_solve, oracle_params, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("conv,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_128_full_parity(conv, tol):
    N, n, Q, bumps = mi.workload("fp32_128")
    f = mi.bump_charge(N, bumps)
    prob = gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, fft_size=96)
    g = gpu_solve(prob, f)
    assert g["info"]["M"] == 96
    prm = oracle_params(g["info"], 3.0, 6.0)
    phi, o = omlc.mlc_solve(f, prm, dgf_cached(Q, prm.Z), keep=True)
    sk = omlc.skeleton_mask(N, n)
    errs = {"phi": rel(g["phi"], phi), "phiB": rel(g["phiB"][sk], o["phiB"][sk]),
            "phiH": rel(g["phiH"], o["phiH"]), "FH": rel(g["FH"], o["FH"]),
            "moments": rel(g["moments"], o["moments"])}
    print(conv, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    if conv == "fp64":
        for k, v in errs.items():
            assert v < tol, (k, v)
    else:
        assert errs["phi"] < tol, errs
        assert errs["moments"] < 1e-12


@pytest.fixture(scope="module")
def big():
    """The 256^3 L27 workload solved by the fp32 and fp64 plans."""
    N, n, Q, bumps = mi.workload("fp32_256_q6")
    f = mi.bump_charge(N, bumps)
    out = {}
    for conv in ("fp64", "fp32"):
        out[conv] = gpu_solve(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv), f)
    return f, out


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
def test_256_coarse_solve_inverts_laplacian(big, conv):
    """Delta^H phi^H = F^H on the interior of the coarse output box
    (convolution with the DGF inverts the stencil, sec. 2 eq. dgf)."""
    f, out = big
    g = out[conv]
    info = g["info"]
    H = info["H"]
    lap = apply_laplacian(g["phiH"], info["Q"], H)
    O_lo, S_lo, No = info["O_lo"], info["S_lo"], info["No"]
    o = O_lo + 1 - S_lo
    F = g["FH"][o:o + No - 2, o:o + No - 2, o:o + No - 2]
    assert rel(lap, F) < 1e-10


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
def test_256_patch_solves_satisfy_stencil(big, conv):
    """phi - h^2 f / 12 satisfies Delta^h u = f at every patch-interior node
    and equals phi^B on the skeleton (sec. 4.1)."""
    f, out = big
    g = out[conv]
    info = g["info"]
    N, n, h = info["N"], info["n"], info["h"]
    u = g["phi"] - h * h / 12.0 * f
    lap = apply_laplacian(u, info["Q"], h)
    inner = ~omlc.skeleton_mask(N, n)[1:-1, 1:-1, 1:-1]
    assert rel(lap[inner], f[1:-1, 1:-1, 1:-1][inner]) < 1e-9
    sk = omlc.skeleton_mask(N, n)
    assert np.abs(u[sk] - g["phiB"][sk]).max() < 1e-14 * np.abs(u).max()


def test_256_fp32_matches_fp64(big):
    """The float32-convolution solve stays within 2e-6 of the float64 one
    (the float64 path matches the oracle to 1e-12 elsewhere)."""
    f, out = big
    assert rel(out["fp32"]["phi"], out["fp64"]["phi"]) < 2e-6
