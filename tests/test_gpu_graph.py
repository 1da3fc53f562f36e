"""A solve captured into a HIP graph by the caller (MI355X only).

The launch sequence of a solve is capture-safe: kernel launches only (no
memsets, no host synchronisation), and the side stream forks from and joins
back into the caller's stream through events, so the whole solve becomes one
graph.  Every replay, with eager solves and synchronisations between the
replays, must equal the eager result bit for bit."""
import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,n,Q,conv", [(32, 8, 4, "fp32"), (64, 16, 6, "fp64")])
def test_graph_replay(N, n, Q, conv):
    import torch
    plan = context().plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, Z=64 if n == 8 else 128))
    f = torch.from_numpy(mi.bump_charge(N, mi.bumps(2, 81))).cuda()
    f2 = torch.from_numpy(mi.bump_charge(N, mi.bumps(3, 82))).cuda()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    ws2 = torch.empty_like(ws)
    phi = torch.empty_like(f)
    phi2 = torch.empty_like(f)
    plan.solve(f, phi, ws)
    plan.solve(f2, phi2, ws2)
    torch.cuda.synchronize()
    ref, ref2 = phi.cpu().numpy(), phi2.cpu().numpy()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):          # the stream's side stream exists before capture
        plan.solve(f, phi, ws, s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.solve(f, phi, ws, s)
    torch.cuda.synchronize()
    for r in range(4):
        phi.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(phi.cpu().numpy(), ref), r
        # eager work between replays, on another workspace
        phi2.fill_(float("nan"))
        plan.solve(f2, phi2, ws2)
        torch.cuda.synchronize()
        assert np.array_equal(phi2.cpu().numpy(), ref2), r
    del g
    torch.cuda.synchronize()
