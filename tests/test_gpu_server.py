"""The serving loop (mlc_server_*) through the C ABI (MI355X only).

Requests of mixed sizes, patch sizes, operators and precisions are queued
while others run; each result must equal the same problem solved alone, bit
for bit (a request's arithmetic does not depend on the launch it shares),
and the oracle's solve of its problem within the bars of the path (float64
convolutions 1e-12, float32 convolutions 2e-6, relative max-norm).  The mix
includes 128^3 requests with 32^3-cell patches and the 27-point operator, the
patch work of the benchmark."""
import os
import time

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import context, rel

pytestmark = pytest.mark.gpu

# (N, n, Q, conv, seed)
MIX = [(32, 8, 4, "fp64", 31), (32, 16, 4, "fp32", 32), (64, 16, 4, "fp32", 33), (32, 8, 6, "fp64", 34),
       (64, 16, 6, "fp32", 35), (128, 32, 6, "fp32", 41), (32, 16, 4, "fp32", 36), (48, 16, 4, "fp32", 37),
       (64, 8, 4, "fp32", 38), (128, 32, 6, "fp64", 42), (32, 16, 4, "fp32", 39), (64, 16, 4, "fp32", 40),
       (128, 32, 6, "fp32", 43)]
TOL = {"fp64": 1e-12, "fp32": 2e-6}


@pytest.fixture(scope="module")
def oracle_phis():
    """The oracle's phi for every request of the mix (default DGF table Z = 128)."""
    out = []
    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        for N, n, Q, conv, s in MIX:
            f = mi.bump_charge(N, mi.bumps(1 + s % 4, s))
            prm = omlc.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=Q, Z=128)
            out.append(omlc.mlc_solve(f, prm, dgf_cached(Q, 128)))
    return out


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


def test_server_mix_equals_alone(oracle_phis):
    import torch
    fs = _charges()
    ref = _alone(fs)
    # the alone solves themselves against the oracle
    for k, (m, r) in enumerate(zip(MIX, ref)):
        e = rel(r, oracle_phis[k])
        print(k, m[:4], f"alone vs oracle {e:.2e}", flush=True)
        assert e < TOL[m[3]], (k, m, e)
    srv = gm.Server(context(), budget_bytes=8 << 30, streams=2, max_batch=8)
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
            assert rel(got, oracle_phis[k]) < TOL[MIX[k][3]], (k, MIX[k])
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


def test_server_autotuned_request_in_tight_arena():
    """A request with an autotuned torus (fft_size = -1) in an arena of
    exactly its host-side workspace figure is admitted and solved, equal to
    the same plan solving alone."""
    import torch
    prob = gm.problem(64, 16, 3.0, 6.0, 4, 4, conv="fp32", fft_size=-1)
    need = gm.problem_workspace_bytes(prob)
    f = torch.from_numpy(mi.bump_charge(64, mi.bumps(2, 44))).cuda()
    plan = context().plan(prob)
    assert plan.workspace_bytes <= need
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    ref = torch.empty_like(f)
    plan.solve(f, ref, ws)
    torch.cuda.synchronize()
    plan.close()
    srv = gm.Server(context(), budget_bytes=need, streams=1, max_batch=2)
    try:
        phis = [torch.empty_like(f) for _ in range(3)]
        torch.cuda.synchronize()
        tickets = [srv.submit(prob, f, p)[1] for p in phis]
        timings = [_wait(srv, t) for t in tickets]
        for tm, p in zip(timings, phis):
            assert tm["status"] == gm.MLC_OK, tm
            assert torch.equal(p, ref)
    finally:
        srv.close()


def test_context_budget_enforced():
    """A context's resident-memory cap refuses a plan (or server arena) that
    would exceed it, and a destroyed plan gives its share back."""
    import torch
    ctx = gm.Context(0, hbm_budget=0)
    try:
        # the DGF table of Z = 64 alone: (129)^3 doubles
        prob = gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64)
        p = ctx.plan(prob)
        p.close()
    finally:
        ctx.close()
    small = gm.Context(0, hbm_budget=129 ** 3 * 8 + 4096)
    try:
        with pytest.raises(gm.MLCError) as ei:
            small.plan(gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64))
        assert ei.value.status == gm.MLC_ERR_OUT_OF_MEMORY
        with pytest.raises(gm.MLCError) as ei:
            gm.Server(small, budget_bytes=1 << 30)
        assert ei.value.status == gm.MLC_ERR_OUT_OF_MEMORY
    finally:
        small.close()
    # plans under a 64 MB cap until one is refused; after closing them the
    # same number fits again
    capped = gm.Context(0, hbm_budget=64 << 20)
    try:
        prob = gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64)
        held = []
        with pytest.raises(gm.MLCError) as ei:
            for _ in range(16):
                held.append(capped.plan(prob))
        assert ei.value.status == gm.MLC_ERR_OUT_OF_MEMORY
        assert 1 <= len(held) < 16
        k = len(held)
        for p in held:
            p.close()
        again = [capped.plan(prob) for _ in range(k)]
        for p in again:
            p.close()
    finally:
        capped.close()
    torch.cuda.synchronize()
