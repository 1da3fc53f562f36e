"""MLC_TRACE (per-call JSON lines of stage times) through the C ABI (MI355X
only): one line per mlc_solve / mlc_solve_batched call with its status,
problems and per-stage device times, including a multilevel plan's coarser
level; the results are those of the untraced calls, and a plan's own
per-kernel timing state is left as it was."""
import json

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu


def test_trace_lines(monkeypatch, tmp_path):
    import torch
    path = tmp_path / "trace.jsonl"
    ctx = context()
    p2 = ctx.plan(gm.problem(64, 16, 3.0, 6.0, 4, 6, conv="fp64"))
    p3 = ctx.plan(gm.problem(64, 8, 3.0, 6.0, 4, 6, conv="fp64", Z=64, levels=3))
    f = torch.from_numpy(mi.smooth_charge(64)).cuda()
    ws = torch.empty(max(p2.workspace_bytes, p3.workspace_bytes), dtype=torch.uint8, device="cuda")
    ref2, ref3 = torch.empty_like(f), torch.empty_like(f)
    p2.solve(f, ref2, ws)
    p3.solve(f, ref3, ws)
    torch.cuda.synchronize()
    monkeypatch.setenv("MLC_TRACE", str(path))
    a, b = torch.empty_like(f), torch.empty_like(f)
    p2.solve(f, a, ws)
    p3.solve(f, b, ws)
    bws = torch.empty(gm.batch_workspace_bytes([p2, p2]), dtype=torch.uint8, device="cuda")
    c, d = torch.empty_like(f), torch.empty_like(f)
    gm.solve_batched([p2, p2], [f, f], [c, d], bws)
    torch.cuda.synchronize()
    monkeypatch.delenv("MLC_TRACE")
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert [x["entry"] for x in lines] == ["mlc_solve", "mlc_solve", "mlc_solve_batched"]
    for x in lines:
        assert x["status"] == "MLC_OK" and x["wall_ms"] > 0
        assert any(k.startswith("conv_") for k in x["stages"])
        assert all(v[0] >= 1 and v[1] >= 0 for v in x["stages"].values())
    assert lines[0]["problems"][0]["N"] == 64 and lines[0]["problems"][0]["levels"] == 2
    assert lines[1]["problems"][0]["levels"] == 3
    assert any(k.startswith("L1.") for k in lines[1]["stages"]), lines[1]["stages"]
    assert len(lines[2]["problems"]) == 2
    for got, ref in ((a, ref2), (b, ref3), (c, ref2), (d, ref2)):
        assert torch.equal(got, ref)
    # the plans' own timing stays off and empty
    assert p2.timing() == {} and p3.timing() == {}
    p2.close()
    p3.close()
