"""The sixth-order variant for the 27-point operator (rhs_order = 6) on
MI355X, through the C ABI: the modified right-hand side f~ of sec. 2 eq.
msCorr (h^4 term from the operator's truncation error, appendix A.1) is
formed on the device and solved with no final correction.

Parity with the oracle (oracle.mlc.mlc_solve_sixth, and the multilevel
solve with rhs_order = 6): f~ itself, F^H, phi^H, phi^B and phi, float64
within 1e-12, float32 convolutions within 2e-6 on phi.  Then the order of
accuracy against the closed-form potential of a smooth radial charge, and
the input check and refusals the variant adds."""
import os

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from oracle.stencils import sixth_order_rhs
from paper_1702_08111_amd import mlc as gm

from gpu_common import _slice, context, gpu_solve, rel

pytestmark = pytest.mark.gpu

CHARGES = {
    "centred": lambda N: mi.poly_charge(N, 10, (0.5, 0.5, 0.5), 0.3),
    "offset": lambda N: mi.poly_charge(N, 6, (0.45, 0.55, 0.5), 0.25),
}


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
@pytest.mark.parametrize("charge", sorted(CHARGES))
def test_sixth_order_parity(charge, conv):
    import torch
    N, n = 32, 8
    f = CHARGES[charge](N)
    prob = gm.problem(N, n, 3.0, 6.0, 4, 6, conv=conv, Z=64, rhs_order=6)
    plan = context().plan(prob)
    g = gpu_solve(prob, f, plan=plan)
    # the modified right-hand side the library formed (the workspace of the
    # solve above was freed; solve again to read it)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    fd = torch.from_numpy(f).cuda()
    phi = torch.empty_like(fd)
    plan.solve(fd, phi, ws)
    torch.cuda.synchronize()
    ft = _slice(ws, plan, gm.MLC_VIEW_CHARGE, torch.float64, (N + 1,) * 3)
    plan.close()
    prm = omlc.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=6, Z=64)
    o_phi, o = omlc.mlc_solve_sixth(f, prm, dgf_cached(6, 64), keep=True)
    sk = omlc.skeleton_mask(N, n)
    errs = {"charge": rel(ft, sixth_order_rhs(f)), "FH": rel(g["FH"], o["FH"]), "phiH": rel(g["phiH"], o["phiH"]),
            "phiB": rel(g["phiB"][sk], o["phiB"][sk]), "phi": rel(g["phi"], o_phi)}
    print(charge, conv, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert errs["charge"] < 1e-14
    if conv == "fp64":
        for k, v in errs.items():
            assert v < 1e-12, (k, v)
    else:
        assert errs["phi"] < 2e-6


def test_sixth_order_multilevel_parity():
    """Three levels with the sixth-order right-hand side at the finest level
    (the coarser levels solve their node charge as before)."""
    import torch
    N, n = 64, 8
    f = CHARGES["offset"](N)
    plan = context().plan(gm.problem(N, n, 3.0, 6.0, 4, 6, conv="fp64", Z=64, levels=3, rhs_order=6))
    fd = torch.from_numpy(f).cuda()
    phi = torch.empty_like(fd)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve(fd, phi, ws)
    torch.cuda.synchronize()
    prm = omlc.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=6, Z=64)
    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        o_phi, _ = omlc.mlc_solve_multilevel(f, prm, 3, dgf_cached(6, 64), rhs_order=6)
    e = rel(phi.cpu().numpy(), o_phi)
    print(f"three levels, rhs_order 6: {e:.2e}", flush=True)
    plan.close()
    assert e < 1e-12


def _closed_form_error(N, rhs_order, conv="fp64"):
    import torch
    f = mi.poly_charge(N)
    ex = mi.poly_potential(N)
    plan = context().plan(gm.problem(N, 32, 3.0, 6.0, 4, 6, conv=conv, rhs_order=rhs_order))
    fd = torch.from_numpy(f).cuda()
    phi = torch.empty_like(fd)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve(fd, phi, ws)
    torch.cuda.synchronize()
    plan.close()
    return float(np.abs(phi.cpu().numpy() - ex).max() / np.abs(ex).max())


def test_sixth_order_convergence():
    """Against the closed form (32^3-cell patches, alpha 3, beta 6): halving h
    divides the sixth-order error by more than 30 and the fourth-order one by
    about 16; at 128^3 the sixth-order solve is more than 100 times more
    accurate."""
    e6 = [_closed_form_error(N, 6) for N in (64, 128)]
    e4 = [_closed_form_error(N, 4) for N in (64, 128)]
    print("sixth order", [f"{e:.3e}" for e in e6], "fourth order", [f"{e:.3e}" for e in e4], flush=True)
    assert e6[0] / e6[1] > 30, e6
    assert 13 < e4[0] / e4[1] < 19, e4
    assert e6[1] < e4[1] / 100


def test_sixth_order_input_check_and_refusals(monkeypatch):
    """With MLC_CHECK=1 a sixth-order plan refuses a charge that is nonzero
    within two nodes of a face (its f~ would reach the boundary), which the
    fourth-order plan accepts; the analytic entry point refuses a
    sixth-order plan."""
    import torch
    N = 32
    f = torch.from_numpy(CHARGES["centred"](N)).cuda()
    bad = f.clone()
    bad[2, 16, 16] = 1e-3
    phi = torch.empty_like(f)
    p6 = context().plan(gm.problem(N, 8, 3.0, 6.0, 4, 6, conv="fp64", Z=64, rhs_order=6))
    p4 = context().plan(gm.problem(N, 8, 3.0, 6.0, 4, 6, conv="fp64", Z=64))
    ws = torch.empty(max(p6.workspace_bytes, p4.workspace_bytes), dtype=torch.uint8, device="cuda")
    monkeypatch.setenv("MLC_CHECK", "1")
    p6.solve(f, phi, ws)
    p4.solve(bad, phi, ws)
    torch.cuda.synchronize()
    with pytest.raises(gm.MLCError) as ei:
        p6.solve(bad, phi, ws)
    assert ei.value.status == gm.MLC_ERR_INVALID_ARG
    monkeypatch.delenv("MLC_CHECK")
    with pytest.raises(gm.MLCError) as ei:
        p6.solve_analytic(mi.smooth_terms(), 2, f.clone(), phi, ws)
    assert ei.value.status == gm.MLC_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    p6.close()
    p4.close()
