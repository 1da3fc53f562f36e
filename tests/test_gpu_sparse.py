"""Skipping empty patches (mlc_problem.skip_empty) on MI355X: a patch whose
node charge is zero has a zero local field and zero moments, so a plan that
skips those patches' local convolutions gives the same phi as one that does
not, equal element for element, in float32 and float64, two and three levels,
the sixth-order variant and a batch that mixes both kinds of plan."""
import time

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

CASES = {
    # (problem keywords, charge)
    "bench_256": (dict(N=256, n=32, alpha=3.0, beta=6.0, P=4, Q=6), lambda: mi.bump_charge(256, mi.workload("fp32_256_q6")[3])),
    "smooth_128_l3": (dict(N=128, n=16, alpha=3.0, beta=6.0, P=4, Q=4, levels=3), lambda: mi.smooth_charge(128)),
    "oscillatory_128": (dict(N=128, n=32, alpha=1.75, beta=3.25, P=4, Q=6, b=3), lambda: mi.oscillatory_charge(128)),
    "sixth_64": (dict(N=64, n=8, alpha=3.0, beta=6.0, P=4, Q=6, Z=64, rhs_order=6),
                 lambda: mi.poly_charge(64, 6, (0.45, 0.55, 0.5), 0.2)),
}


def _solve(plan, f, reps=1):
    import torch
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.full_like(f, np.nan)
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    return phi, (time.perf_counter() - t0) * 1e3 / reps


@pytest.mark.parametrize("conv", ["fp32", "fp64"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_skip_empty_equals_dense(name, conv):
    import torch
    kw, charge = CASES[name]
    f = torch.from_numpy(charge()).cuda()
    dense = context().plan(gm.problem(conv=conv, **kw))
    sparse = context().plan(gm.problem(conv=conv, skip_empty=1, **kw))
    reps = 10 if name == "bench_256" else 2
    a, ta = _solve(dense, f, reps)
    b, tb = _solve(sparse, f, reps)
    print(f"{name} {conv}: dense {ta:.3f} ms, skipping empty patches {tb:.3f} ms", flush=True)
    assert torch.equal(a, b)
    dense.close()
    sparse.close()


def test_batch_mixing_skip_and_dense():
    import torch
    ctx = context()
    kws = [dict(N=64, n=16, alpha=3.0, beta=6.0, P=4, Q=4), dict(N=64, n=16, alpha=3.0, beta=6.0, P=4, Q=4, skip_empty=1),
           dict(N=96, n=16, alpha=3.0, beta=6.0, P=4, Q=4, skip_empty=1)]
    fs = [torch.from_numpy(mi.bump_charge(k["N"], mi.bumps(1, 60 + i, radius=(0.1, 0.15)))).cuda()
          for i, k in enumerate(kws)]
    plans = [ctx.plan(gm.problem(conv="fp32", **k)) for k in kws]
    alone = [_solve(ctx.plan(gm.problem(conv="fp32", **dict(k, skip_empty=0))), f)[0] for k, f in zip(kws, fs)]
    ws = torch.empty(gm.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    phis = [torch.full_like(f, np.nan) for f in fs]
    gm.solve_batched(plans, fs, phis, ws)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(phis, alone)):
        assert torch.equal(x, y), k
    for p in plans:
        p.close()
