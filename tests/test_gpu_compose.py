"""The features together through the C ABI (MI355X only): multilevel plans
(with per-level radii), sixth-order plans, a box domain with empty patches
skipped and plain two-level plans in one
batched call, in a library-captured batch graph, through the serving loop
and on the static scratch; every result equals the same plan solving alone,
bit for bit (a problem's arithmetic does not depend on what shares its
launch)."""
import time

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

PROBLEMS = [
    # (problem keywords, charge)
    (dict(N=64, n=8, alpha=3.0, beta=6.0, P=4, Q=6, Z=64, levels=3), lambda: mi.smooth_charge(64)),
    (dict(N=64, n=8, alpha=2.0, beta=3.0, P=4, Q=6, Z=64, levels=3, level_alpha=(3.0,), rhs_order=6),
     lambda: mi.poly_charge(64, 6, (0.45, 0.55, 0.5), 0.25)),
    (dict(N=32, n=8, alpha=3.0, beta=6.0, P=4, Q=6, Z=64, rhs_order=6), lambda: mi.poly_charge(32)),
    (dict(N=32, n=8, alpha=3.0, beta=6.0, P=4, Q=4, Z=64), lambda: mi.bump_charge(32, mi.bumps(2, 5))),
    (dict(N=128, n=16, alpha=3.0, beta=6.0, P=4, Q=4, Z=128, levels=3), lambda: mi.smooth_charge(128)),
    # a box domain with empty patches skipped
    (dict(N=(64, 48, 32), n=16, alpha=3.0, beta=6.0, P=4, Q=4, Z=128, skip_empty=1), lambda: _box_charge((64, 48, 32))),
]


def _box_charge(B):
    h = 1.0 / max(B)
    g = [np.arange(b + 1) * h for b in B]
    r = np.sqrt((g[0][:, None, None] - 0.45) ** 2 + (g[1][None, :, None] - 0.35) ** 2
                + (g[2][None, None, :] - 0.25) ** 2) / 0.2
    return np.where(r < 1.0, (1.0 - r * r) ** 4, 0.0)


def _setup(conv):
    import torch
    ctx = context()
    plans = [ctx.plan(gm.problem(conv=conv, **kw)) for kw, _ in PROBLEMS]
    fs = [torch.from_numpy(ch()).cuda() for _, ch in PROBLEMS]
    alone = []
    for p, f in zip(plans, fs):
        ws = torch.empty(p.workspace_bytes, dtype=torch.uint8, device="cuda")
        phi = torch.empty_like(f)
        p.solve(f, phi, ws)
        torch.cuda.synchronize()
        alone.append(phi.clone())
    return plans, fs, alone


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
def test_batch_and_graph_equal_alone(conv):
    import torch
    plans, fs, alone = _setup(conv)
    ws = torch.empty(gm.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    phis = [torch.full_like(f, np.nan) for f in fs]
    gm.solve_batched(plans, fs, phis, ws)
    torch.cuda.synchronize()
    for k, (a, b) in enumerate(zip(phis, alone)):
        assert torch.equal(a, b), (k, PROBLEMS[k][0])
    g = gm.BatchGraph(plans, fs, phis, ws)
    try:
        for rep in range(3):
            for x in phis:
                x.fill_(np.nan)
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(phis, alone)):
                assert torch.equal(a, b), (rep, k)
            # eager work between the replays
            solo = torch.empty_like(fs[0])
            plans[0].solve(fs[0], solo, ws)
            torch.cuda.synchronize()
            assert torch.equal(solo, alone[0])
    finally:
        g.close()
    for p in plans:
        p.close()


def test_server_equals_alone():
    import torch
    _, fs, alone = _setup("fp32")
    srv = gm.Server(context(), budget_bytes=4 << 30, streams=2, max_batch=4)
    try:
        phis = [torch.full_like(f, np.nan) for f in fs]
        torch.cuda.synchronize()
        tickets = []
        for (kw, _), f, phi in zip(PROBLEMS, fs, phis):
            st, t = srv.submit(gm.problem(conv="fp32", **kw), f, phi)
            assert st == gm.MLC_OK
            tickets.append(t)
        t0 = time.time()
        for t in tickets:
            while srv.poll(t) is None:
                assert time.time() - t0 < 120, "request did not finish"
                time.sleep(0.001)
        srv.drain()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(phis, alone)):
            assert torch.equal(a, b), (k, PROBLEMS[k][0])
    finally:
        srv.close()


def test_static_scratch_multilevel_and_sixth_order():
    """mlc_solve_static on plans whose workspace fits the static scratch."""
    import torch
    plans, fs, alone = _setup("fp32")
    done = 0
    for p, f, ref in zip(plans, fs, alone):
        if p.workspace_bytes > gm.MLC_STATIC_SCRATCH_BYTES:
            continue
        phi = torch.full_like(f, np.nan)
        p.solve_static(f, phi)
        torch.cuda.synchronize()
        assert torch.equal(phi, ref)
        done += 1
    assert done >= 3
    for p in plans:
        p.close()
