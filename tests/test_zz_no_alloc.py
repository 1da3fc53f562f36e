"""mlc_solve_static, the allocation-free solve on the library's static
scratch (MI355X only), against mlc_solve with a caller workspace: two calls
in a row on one stream, the second with a smaller problem (so the scratch
still holds the first call's values), each equal to the workspace solve bit
for bit and within the path's bars of it (float64 1e-12, float32 2e-6,
relative max-norm).  A plan whose workspace exceeds the scratch is refused
before anything is enqueued."""
import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context, rel

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-6}


def _workspace_solve(plan, f):
    import torch
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.empty_like(f)
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    del ws
    return phi


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
def test_static_equals_workspace_solve(conv):
    import torch
    ctx = context()
    # first the larger problem, then a smaller one over the same scratch
    cases = [(64, 16, 6, 0, mi.bumps(3, 51, radius=(0.1, 0.2))), (32, 8, 4, 0, mi.bumps(2, 52, radius=(0.1, 0.25)))]
    plans, fs = [], []
    for N, n, Q, fft, b in cases:
        plan = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, fft_size=fft))
        assert plan.workspace_bytes <= gm.MLC_STATIC_SCRATCH_BYTES
        plans.append(plan)
        fs.append(torch.from_numpy(mi.bump_charge(N, b)).cuda())
    assert plans[1].workspace_bytes < plans[0].workspace_bytes
    refs = [_workspace_solve(p, f) for p, f in zip(plans, fs)]
    stream = torch.cuda.current_stream()
    outs = [torch.full_like(f, np.nan) for f in fs]
    torch.cuda.synchronize()
    for p, f, o in zip(plans, fs, outs):
        p.solve_static(f, o, stream)
    torch.cuda.synchronize()
    for k, (o, r) in enumerate(zip(outs, refs)):
        e = rel(o.cpu().numpy(), r.cpu().numpy())
        print(conv, cases[k][:3], f"static vs workspace {e:.2e}, bitwise {torch.equal(o, r)}", flush=True)
        assert e < TOL[conv], (k, e)
        assert torch.equal(o, r), k
    # once more in reverse order: the larger problem over the smaller one's leftovers
    outs2 = [torch.full_like(f, np.nan) for f in fs]
    torch.cuda.synchronize()
    for k in (1, 0):
        plans[k].solve_static(fs[k], outs2[k], stream)
    torch.cuda.synchronize()
    for o, r in zip(outs2, refs):
        assert torch.equal(o, r)
    for p in plans:
        p.close()


def test_static_refuses_a_plan_beyond_the_scratch():
    import torch
    ctx = context()
    plan = ctx.plan(gm.problem(128, 16, 3.0, 6.0, 4, 4, conv="fp32", fft_size=96))
    try:
        assert plan.workspace_bytes > gm.MLC_STATIC_SCRATCH_BYTES
        f = torch.zeros((129,) * 3, dtype=torch.float64, device="cuda")
        phi = torch.full_like(f, 7.0)
        torch.cuda.synchronize()
        with pytest.raises(gm.MLCError) as ei:
            plan.solve_static(f, phi)
        assert ei.value.status == gm.MLC_ERR_UNSUPPORTED
        torch.cuda.synchronize()
        assert bool((phi == 7.0).all())   # nothing was enqueued
    finally:
        plan.close()
