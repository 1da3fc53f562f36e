"""GPU parity against the oracle, through the C ABI (MI355X only).

Bars: float64 path within 1e-12 relative max-norm of the oracle; float32
local convolutions within 2e-6 on phi (every other stage is float64)."""
import numpy as np
import pytest

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import context, gpu_solve, oracle_local, oracle_params, rel

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-6


@pytest.mark.parametrize("Q", [4, 6])
def test_dgf_table(Q):
    """The GPU's DGF (DST-I Dirichlet solve, appendix A.1) equals the oracle's."""
    import torch
    ctx = context()
    Z = 64
    ptr = ctx.dgf_table(Q, Z)
    W = 2 * Z + 1
    t = torch.empty(W ** 3, dtype=torch.float64, device="cuda")
    # copy through torch from the raw device pointer
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    assert hip.hipMemcpy(ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(ptr), W ** 3 * 8, 3) == 0
    g = t.cpu().numpy().reshape(W, W, W)
    o = dgf_cached(Q, Z)
    assert rel(g, o) < 1e-13


def _case(name):
    cases = {
        # (N, n, alpha, beta, P, Q, fft, Z, bumps)
        "plain32": (32, 8, 3.0, 6.0, 4, 4, 0, 64, mi.one_bump()),
        "plain32_q6": (32, 8, 3.0, 6.0, 4, 6, 0, 64, mi.bumps(2, 7, radius=(0.15, 0.25))),
        "mlc0_32": (32, 8, 3.0, 3.0, 4, 4, 0, 64, mi.bumps(2, 8, radius=(0.15, 0.25))),
        "p1_32": (32, 8, 3.0, 6.0, 1, 4, 0, 64, mi.bumps(3, 9, radius=(0.1, 0.2))),
        "ragged48": (48, 16, 3.0, 6.0, 4, 4, 90, 128, mi.bumps(2, 11, radius=(0.12, 0.2))),
        # one patch: every neighbour lattice is empty, the skeleton is the box surface
        "single16": (16, 16, 3.0, 6.0, 4, 4, 0, 128, mi.bumps(2, 12, radius=(0.15, 0.3))),
        # 4 and 10 Legendre modes (moment slices of 4 padded with zeros)
        "p2_32": (32, 8, 3.0, 6.0, 2, 4, 0, 64, mi.bumps(2, 13, radius=(0.1, 0.25))),
        "p3_32": (32, 8, 3.0, 6.0, 3, 4, 0, 64, mi.bumps(2, 14, radius=(0.1, 0.25))),
        # the smallest and largest coplanar interpolation radius (output boxes
        # of widths Wa + 2 and Wa + 8, tori 50 and 72)
        "b1_32": (32, 8, 3.0, 6.0, 4, 4, 0, 64, mi.bumps(2, 15, radius=(0.1, 0.25))),
        "b4_32": (32, 8, 3.0, 6.0, 4, 6, 0, 64, mi.bumps(2, 16, radius=(0.1, 0.25))),
        # the benchmark's patch work (32^3-cell patches, L27, M = 160, far-field
        # torus 250, Z = 128) on 2^3 patches
        "n32_64": (64, 32, 3.0, 6.0, 4, 6, 160, 128, mi.bumps(2, 17, radius=(0.1, 0.2))),
        # P >= 5: 35, 56 and 165 Legendre modes, projected with the full Boole
        # Gram matrix
        "p5_32": (32, 8, 3.0, 6.0, 5, 4, 0, 64, mi.bumps(2, 18, radius=(0.1, 0.25))),
        "p6_32_q6": (32, 8, 3.0, 6.0, 6, 6, 0, 64, mi.bumps(2, 19, radius=(0.1, 0.25))),
        "p9_32": (32, 8, 3.0, 6.0, 9, 4, 0, 64, mi.bumps(2, 20, radius=(0.1, 0.25))),
        # the parameters of the paper's Table 7 (L27, alpha 1.75, beta 3.25,
        # P = 9) with 32^3-cell patches
        "t7_64": (64, 32, 1.75, 3.25, 9, 6, 0, 128, mi.bumps(2, 21, radius=(0.1, 0.2))),
        # beta margins below 4b (d_beta / 4 < b): the coarse output box starts
        # below the right-hand side's box, its torus slots wrap around
        "mlc0_32_q6": (32, 8, 3.0, 3.0, 4, 6, 0, 64, mi.bumps(2, 22, radius=(0.1, 0.25))),
        "narrow_beta_q6": (32, 8, 2.0, 3.0, 4, 6, 0, 64, mi.bumps(2, 23, radius=(0.1, 0.25))),
        "mlc0_64_n16": (64, 16, 2.0, 2.0, 4, 6, 0, 64, mi.bumps(2, 24, radius=(0.1, 0.2))),
        # the smallest inner radius: Omega_alpha is the patch itself (d_alpha = 0)
        "alpha1_32": (32, 8, 1.0, 3.0, 4, 4, 0, 64, mi.bumps(2, 25, radius=(0.1, 0.25))),
        "mlc0_alpha1_32": (32, 8, 1.0, 1.0, 4, 6, 0, 64, mi.bumps(2, 26, radius=(0.1, 0.25))),
    }
    return cases[name]


# interpolation radius b of a case (0: the default Q/2)
B_OF = {"b1_32": 1, "b4_32": 4}


def _check_all(name, conv):
    N, n, alpha, beta, P, Q, fft, Z, bumps = _case(name)
    f = mi.bump_charge(N, bumps)
    prob = gm.problem(N, n, alpha, beta, P, Q, b=B_OF.get(name, 0), conv=conv, fft_size=fft, Z=Z)
    g = gpu_solve(prob, f)
    prm = oracle_params(g["info"], alpha, beta)
    phi, o = omlc.mlc_solve(f, prm, dgf_cached(Q, Z), keep=True)
    sk = omlc.skeleton_mask(N, n)
    errs = {
        "moments": rel(g["moments"], o["moments"]),
        "FH": rel(g["FH"], o["FH"]),
        "phiH": rel(g["phiH"], o["phiH"]),
        "phiB": rel(g["phiB"][sk], o["phiB"][sk]),
        "phi": rel(g["phi"], phi),
    }
    # local fields of a few patches, including corners of the patch lattice
    ppa = N // n
    for i in [(0, 0, 0), (ppa - 1, ppa // 2, 0), (ppa // 2, ppa // 2, ppa // 2)]:
        pidx = (i[0] * ppa + i[1]) * ppa + i[2]
        c, dl = oracle_local(prm, f, i)
        errs[f"coarse{i}"] = rel(g["local_coarse"][pidx], c)
        errs[f"delta{i}"] = rel(g["local_delta"][pidx], dl)
    print(name, conv, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    return errs


@pytest.mark.parametrize("name", ["plain32", "plain32_q6", "mlc0_32", "p1_32", "ragged48", "single16", "p2_32",
                                  "p3_32", "b1_32", "b4_32", "n32_64", "p5_32", "p6_32_q6", "p9_32", "t7_64",
                                  "mlc0_32_q6", "narrow_beta_q6", "mlc0_64_n16", "alpha1_32", "mlc0_alpha1_32"])
def test_fp64_parity(name):
    errs = _check_all(name, "fp64")
    for k, v in errs.items():
        assert v < TOL64, (k, v)


@pytest.mark.parametrize("name", ["plain32", "plain32_q6", "mlc0_32", "p1_32", "ragged48", "single16", "b1_32",
                                  "b4_32", "n32_64", "p5_32", "p9_32", "mlc0_32_q6"])
def test_fp32_parity(name):
    errs = _check_all(name, "fp32")
    assert errs["phi"] < TOL32, errs
    assert errs["moments"] < TOL64


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
def test_zero_charge_gives_zero(conv):
    """Degenerate input: f = 0 gives phi = 0 exactly (every stage is linear)."""
    f = np.zeros((33, 33, 33))
    g = gpu_solve(gm.problem(32, 8, 3.0, 6.0, 4, 4, conv=conv, Z=64), f, keep=False)
    assert np.array_equal(g["phi"], np.zeros_like(f))


def test_linearity():
    """phi(2 f1 - 3 f2) = 2 phi(f1) - 3 phi(f2) to rounding (float64 path)."""
    prob = gm.problem(48, 16, 3.0, 6.0, 4, 4, conv="fp64")
    f1 = mi.bump_charge(48, mi.bumps(2, 31))
    f2 = mi.bump_charge(48, mi.bumps(3, 32))
    p1 = gpu_solve(prob, f1, keep=False)["phi"]
    p2 = gpu_solve(prob, f2, keep=False)["phi"]
    p3 = gpu_solve(prob, 2 * f1 - 3 * f2, keep=False)["phi"]
    assert rel(p3, 2 * p1 - 3 * p2) < 1e-13
