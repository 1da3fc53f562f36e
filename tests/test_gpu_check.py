"""The optional input check (MLC_CHECK=1) through the C ABI (MI355X only):
a charge that is nonzero on the outer boundary (the method needs its support
inside the domain, sec. 4) is rejected before anything is enqueued, on any
of the six faces; a valid charge passes; without the variable nothing is
checked."""
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu


def test_boundary_check(monkeypatch):
    import torch
    N = 32
    plan = context().plan(gm.problem(N, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64))
    f = torch.from_numpy(mi.bump_charge(N, mi.one_bump())).cuda()
    phi = torch.empty_like(f)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    monkeypatch.setenv("MLC_CHECK", "1")
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    for node in [(0, 5, 7), (N, 3, 3), (9, 0, 2), (4, N, 30), (1, 2, 0), (N, N, N)]:
        bad = f.clone()
        bad[node] = 1e-3
        with pytest.raises(gm.MLCError) as ei:
            plan.solve(bad, phi, ws)
        assert ei.value.status == gm.MLC_ERR_INVALID_ARG, node
        with pytest.raises(gm.MLCError):
            gm.solve_batched([plan, plan], [f, bad], [phi, torch.empty_like(f)],
                             torch.empty(gm.batch_workspace_bytes([plan, plan]), dtype=torch.uint8, device="cuda"))
    monkeypatch.delenv("MLC_CHECK")
    bad = f.clone()
    bad[0, 0, 0] = 1e-3
    plan.solve(bad, phi, ws)   # unchecked: accepted
    torch.cuda.synchronize()
