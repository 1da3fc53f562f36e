"""The serving loop (mlc_server_*) through the C ABI (MI355X only).

Requests of mixed sizes, patch sizes, operators and precisions are queued
while others run; each result must equal the same problem solved alone, bit
for bit (a request's arithmetic does not depend on the launch it shares)."""
import time

import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

# (N, n, Q, conv, seed)
MIX = [(32, 8, 4, "fp64", 31), (32, 16, 4, "fp32", 32), (64, 16, 4, "fp32", 33), (32, 8, 6, "fp64", 34),
       (64, 16, 6, "fp32", 35), (32, 16, 4, "fp32", 36), (48, 16, 4, "fp32", 37), (64, 8, 4, "fp32", 38),
       (32, 16, 4, "fp32", 39), (64, 16, 4, "fp32", 40)]


def _problem(N, n, Q, conv):
    return gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv)


def _charges():
    import torch
    return [torch.from_numpy(mi.bump_charge(N, mi.bumps(1 + s % 4, s))).cuda() for N, _, _, _, s in MIX]


def _alone(fs):
    import torch
    out = []
    for (N, n, Q, conv, _), f in zip(MIX, fs):
        plan = context().plan(_problem(N, n, Q, conv))
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        phi = torch.empty_like(f)
        plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        out.append(phi.cpu().numpy())
        plan.close()
    return out


def _wait(srv, ticket, timeout=120.0):
    t0 = time.time()
    while True:
        r = srv.poll(ticket)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, "request did not finish"
        time.sleep(0.001)


def test_server_mix_equals_alone():
    import torch
    fs = _charges()
    ref = _alone(fs)
    srv = gm.Server(context(), budget_bytes=4 << 30, streams=2, max_batch=8)
    try:
        phis = [torch.full_like(f, np.nan) for f in fs]
        torch.cuda.synchronize()   # the server's streams must not race the fill
        half = len(MIX) // 2
        tickets = []
        for k in range(half):
            st, t = srv.submit(_problem(*MIX[k][:4]), fs[k], phis[k])
            assert st == gm.MLC_OK
            tickets.append(t)
        # the rest arrive while the first ones are queued or running
        time.sleep(0.05)
        for k in range(half, len(MIX)):
            st, t = srv.submit(_problem(*MIX[k][:4]), fs[k], phis[k])
            assert st == gm.MLC_OK
            tickets.append(t)
        timings = [_wait(srv, t) for t in tickets]
        srv.drain()
        torch.cuda.synchronize()
        for k, tm in enumerate(timings):
            assert tm["status"] == gm.MLC_OK, (k, tm)
            assert tm["batch_size"] >= 1 and tm["device_ms"] > 0
            assert 0 <= tm["queue_ms"] <= tm["total_ms"]
            got = phis[k].cpu().numpy()
            assert np.array_equal(got, ref[k]), (k, MIX[k], float(np.nanmax(np.abs(got - ref[k]))))
        print("batch sizes", [tm["batch_size"] for tm in timings], flush=True)
        assert max(tm["batch_size"] for tm in timings) > 1
        # a released ticket is unknown afterwards
        with pytest.raises(gm.MLCError):
            srv.poll(tickets[0])
    finally:
        srv.close()


def test_server_tight_budget():
    """An arena that fits one request at a time still finishes the stream in
    order with the same results; a request larger than the arena is refused."""
    import torch
    fs = _charges()
    ref = _alone(fs)
    biggest = max(gm.problem_workspace_bytes(_problem(*m[:4])) for m in MIX)
    srv = gm.Server(context(), budget_bytes=biggest, streams=2, max_batch=4)
    try:
        phis = [torch.empty_like(f) for f in fs]
        torch.cuda.synchronize()
        tickets = []
        for k, m in enumerate(MIX):
            st, t = srv.submit(_problem(*m[:4]), fs[k], phis[k])
            assert st == gm.MLC_OK
            tickets.append(t)
        big = _problem(256, 32, 6, "fp32")
        assert gm.problem_workspace_bytes(big) > biggest
        with pytest.raises(gm.MLCError) as ei:
            srv.submit(big, fs[0], phis[0])
        assert ei.value.status == gm.MLC_ERR_OUT_OF_MEMORY
        srv.drain()
        for k, t in enumerate(tickets):
            tm = srv.poll(t)
            assert tm is not None and tm["status"] == gm.MLC_OK
            assert np.array_equal(phis[k].cpu().numpy(), ref[k]), k
    finally:
        srv.close()


def test_server_queue_limit():
    """With max_queue = 1 a second request is refused (MLC_ERR_BUSY) while the
    first is unfinished (the server builds its plan on first use, which takes
    far longer than a submit), and accepted after."""
    import torch
    srv = gm.Server(context(), budget_bytes=1 << 30, streams=1, max_batch=1, max_queue=1)
    try:
        f = torch.from_numpy(mi.bump_charge(32, mi.one_bump())).cuda()
        phi = torch.empty_like(f)
        phi2 = torch.empty_like(f)
        torch.cuda.synchronize()
        prob = gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64")
        st, t1 = srv.submit(prob, f, phi)
        assert st == gm.MLC_OK
        st, _ = srv.submit(prob, f, phi2)
        assert st == gm.MLC_ERR_BUSY
        tm = _wait(srv, t1)
        assert tm["status"] == gm.MLC_OK
        st, t2 = srv.submit(prob, f, phi2)
        assert st == gm.MLC_OK
        assert _wait(srv, t2)["status"] == gm.MLC_OK
        assert np.array_equal(phi.cpu().numpy(), phi2.cpu().numpy())
    finally:
        srv.close()
