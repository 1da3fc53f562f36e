"""Solves on caller streams (MI355X only).

A solve forks part of its work onto a side stream of the caller's stream and
joins back before its last stages, so solves enqueued back to back on one
stream may share a workspace, and solves on different streams (each with its
own workspace) run independently.  Every result must equal the same solve
run alone, bit for bit."""
import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu


def _charges(N, seeds):
    import torch
    return [torch.from_numpy(mi.bump_charge(N, mi.bumps(2, s))).cuda() for s in seeds]


def _alone(plan, f):
    import torch
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.empty_like(f)
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


@pytest.mark.parametrize("conv", ["fp32", "fp64"])
def test_back_to_back_one_workspace(conv):
    """Four solves of different charges on one non-default stream, one
    workspace, no host synchronisation between them: each solve's first
    kernels overwrite workspace that the previous solve's side stream read."""
    import torch
    plan = context().plan(gm.problem(96, 16, 3.0, 6.0, 4, 4, conv=conv))
    fs = _charges(96, [61, 62, 63, 64])
    ref = [_alone(plan, f) for f in fs]
    s = torch.cuda.Stream()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phis = [torch.full_like(f, np.nan) for f in fs]
    torch.cuda.synchronize()
    for f, phi in zip(fs, phis):
        plan.solve(f, phi, ws, s)
    s.synchronize()
    for k in range(len(fs)):
        got = phis[k].cpu().numpy()
        assert np.array_equal(got, ref[k]), (conv, k, float(np.nanmax(np.abs(got - ref[k]))))


def test_two_streams_interleaved():
    """Solves alternating between two caller streams (each stream its own
    workspace and side stream) equal the same solves run one at a time."""
    import torch
    plan = context().plan(gm.problem(96, 16, 3.0, 6.0, 4, 6, conv="fp32"))
    fs = _charges(96, [71, 72, 73, 74, 75, 76])
    ref = [_alone(plan, f) for f in fs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    wss = [torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda") for _ in streams]
    phis = [torch.full_like(f, np.nan) for f in fs]
    torch.cuda.synchronize()
    for k, (f, phi) in enumerate(zip(fs, phis)):
        plan.solve(f, phi, wss[k % 2], streams[k % 2])
    for s in streams:
        s.synchronize()
    for k in range(len(fs)):
        assert np.array_equal(phis[k].cpu().numpy(), ref[k]), k
