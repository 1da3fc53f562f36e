"""Batched solves of uneven problems through the C ABI (MI355X only).

Problems whose patch work is identical (patch size, radii, P, Q, b, local
torus, precision) share every patch-level launch; each result must be the
same bit for bit as the problem solved alone, and match the oracle to the
single-solve bars."""
import numpy as np
import pytest

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import context, oracle_params, rel

pytestmark = pytest.mark.gpu


class Plans:
    def __init__(self):
        self.cache = {}

    def get(self, N, n, Q, conv, Z=128):
        key = (N, n, Q, conv, Z)
        if key not in self.cache:
            self.cache[key] = context().plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, Z=Z))
        return self.cache[key]


def _alone(plan, f):
    import torch
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.empty_like(f)
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    return phi.cpu().numpy()


def _batch(plans, fs):
    import torch
    ws = torch.empty(gm.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    phis = [torch.empty_like(f) for f in fs]
    gm.solve_batched(plans, fs, phis, ws)
    torch.cuda.synchronize()
    return [p.cpu().numpy() for p in phis]


def test_batch_mixed_classes():
    """Two classes interleaved (n=16 float32, n=8 float64), three grid sizes."""
    import torch
    P = Plans()
    spec = [(32, 16, "fp32", mi.bumps(2, 21)), (32, 8, "fp64", mi.bumps(1, 22, radius=(0.15, 0.25))),
            (64, 16, "fp32", mi.bumps(3, 23)), (48, 16, "fp32", mi.bumps(2, 24)),
            (32, 16, "fp32", mi.bumps(4, 25)), (32, 8, "fp64", mi.bumps(2, 26, radius=(0.15, 0.25)))]
    plans = [P.get(N, n, 4, conv) for N, n, conv, _ in spec]
    fs_np = [mi.bump_charge(N, b) for N, _, _, b in spec]
    fs = [torch.from_numpy(f).cuda() for f in fs_np]
    got = _batch(plans, fs)
    for k, (N, n, conv, b) in enumerate(spec):
        alone = _alone(plans[k], fs[k])
        assert np.array_equal(got[k], alone), (k, N, n, conv, rel(got[k], alone))
    for k in (0, 1):
        N, n, conv, _ = spec[k]
        prm = oracle_params(plans[k].info, 3.0, 6.0)
        ref = omlc.mlc_solve(fs_np[k], prm, dgf_cached(4, 128))
        e = rel(got[k], ref)
        print(k, N, n, conv, f"{e:.2e}", flush=True)
        assert e < (2e-6 if conv == "fp32" else 1e-12)


def test_batch_uneven_64():
    """The 64-problem uneven batch (N in {32..192}, 16^3-cell patches, L19,
    float32 convolutions): every result equals its solve alone; the N=32
    members match the oracle."""
    import torch
    P = Plans()
    probs = mi.batch_problems()
    plans = [P.get(N, 16, 4, "fp32") for N, _ in probs]
    fs = [torch.from_numpy(mi.bump_charge(N, b)).cuda() for N, b in probs]
    got = _batch(plans, fs)
    print("patches", sum(p.info["npatch"] for p in plans), flush=True)
    for k in range(len(probs)):
        alone = _alone(plans[k], fs[k])
        assert np.array_equal(got[k], alone), (k, probs[k][0], rel(got[k], alone))
    small = [k for k, (N, _) in enumerate(probs) if N == 32][:2]
    assert small
    for k in small:
        prm = oracle_params(plans[k].info, 3.0, 6.0)
        ref = omlc.mlc_solve(fs[k].cpu().numpy(), prm, dgf_cached(4, 128))
        e = rel(got[k], ref)
        print(k, f"{e:.2e}", flush=True)
        assert e < 2e-6


def test_batch_validation():
    """A batch call rejects a short workspace before enqueueing anything."""
    import torch
    P = Plans()
    plans = [P.get(32, 16, 4, "fp32"), P.get(32, 8, 4, "fp64")]
    fs = [torch.zeros((33,) * 3, dtype=torch.float64, device="cuda") for _ in plans]
    phis = [torch.empty_like(f) for f in fs]
    need = gm.batch_workspace_bytes(plans)
    ws = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(gm.MLCError):
        gm.solve_batched(plans, fs, phis, ws)


def test_autotuned_torus():
    """fft_size = -1 picks one of the built tori >= the Hockney minimum (the
    same one again from the context's cache) and the solve keeps parity."""
    import torch
    ctx = context()
    prob = gm.problem(64, 16, 3.0, 6.0, 4, 4, conv="fp32", fft_size=-1)
    p1 = ctx.plan(prob)
    p2 = ctx.plan(prob)
    M, zpb = p1.info["M"], p1.info["out_planes"]
    print("autotuned M", M, "output planes per block", zpb, flush=True)
    assert M in (90, 96, 120, 128) and p2.info["M"] == M and p2.info["out_planes"] == zpb
    assert zpb in (1, 2, 3, 5, 8)
    f_np = mi.bump_charge(64, mi.bumps(2, 41))
    f = torch.from_numpy(f_np).cuda()
    got = _alone(p1, f)
    prm = oracle_params(p1.info, 3.0, 6.0)
    ref = omlc.mlc_solve(f_np, prm, dgf_cached(4, 128))
    assert rel(got, ref) < 2e-6
    # the planes per block decide which block computes an output plane, not
    # how: the plan of the same torus with the default tiling gives the same
    # result bit for bit
    p3 = ctx.plan(gm.problem(64, 16, 3.0, 6.0, 4, 4, conv="fp32", fft_size=M))
    assert p3.info["out_planes"] == (5 if M >= 150 else 1)
    assert np.array_equal(_alone(p3, f), got)
    p1.close()
    p2.close()
    p3.close()


@pytest.mark.parametrize("conv", ["fp32", "fp64"])
def test_batch_graph_replay(conv):
    """A batch of two classes captured once by the library (mlc_graph_create)
    and replayed: every replay equals the eager batched solve bit for bit,
    with eager work and synchronisations between replays, and a replay reads
    the charges' current contents."""
    import torch
    P = Plans()
    spec = [(32, 16, mi.bumps(2, 61)), (48, 16, mi.bumps(3, 62)), (32, 8, mi.bumps(2, 63, radius=(0.15, 0.25))),
            (64, 16, mi.bumps(1, 64))]
    plans = [P.get(N, n, 4, conv) for N, n, _ in spec]
    fs = [torch.from_numpy(mi.bump_charge(N, b)).cuda() for N, _, b in spec]
    fs2 = [torch.from_numpy(mi.bump_charge(N, mi.bumps(2, 70 + k))).cuda() for k, (N, _, _) in enumerate(spec)]
    ref = _batch(plans, fs)
    ref2 = _batch(plans, fs2)
    ws = torch.empty(gm.batch_workspace_bytes(plans), dtype=torch.uint8, device="cuda")
    phis = [torch.empty_like(f) for f in fs]
    src = [f.clone() for f in fs]
    torch.cuda.synchronize()
    g = gm.BatchGraph(plans, src, phis, ws)
    try:
        for r in range(4):
            for p in phis:
                p.fill_(float("nan"))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            for k in range(len(spec)):
                assert np.array_equal(phis[k].cpu().numpy(), ref[k]), (r, k)
            # eager work between replays, on its own workspace
            assert all(np.array_equal(a, b) for a, b in zip(_batch(plans, fs2), ref2))
        # new charges in the same arrays: the replay solves them
        for a, b in zip(src, fs2):
            a.copy_(b)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        for k in range(len(spec)):
            assert np.array_equal(phis[k].cpu().numpy(), ref2[k]), k
    finally:
        g.close()
    torch.cuda.synchronize()
