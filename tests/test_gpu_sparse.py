"""Skipping empty patches (mlc_problem.skip_empty) on MI355X: a patch whose
node charge is zero has a zero local field and zero moments, so a plan that
skips those patches' local convolutions gives the same phi as one that does
not, equal element for element, in float32 and float64, two and three levels,
the sixth-order variant and a batch that mixes both kinds of plan; and plans
that hold per-patch buffers for the live patches only (max_live)."""
import time

import numpy as np
import pytest

import mlc_inputs as mi
from oracle.stencils import sixth_order_rhs
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
    "bumps_128_l3": (dict(N=128, n=16, alpha=3.0, beta=6.0, P=4, Q=4, levels=3),
                     lambda: mi.bump_charge(128, mi.bumps(2, 81, radius=(0.1, 0.15)))),
    # the 2048^3 runs' settings (sec. 7.2, Table 14) on a smaller grid
    "oscillatory_512_l4": (dict(N=512, n=32, alpha=1.75, beta=3.25, P=4, Q=6, b=3, levels=4, level_alpha=(2.0, 2.25)),
                           lambda: mi.oscillatory_charge(512)),
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


def _live_count(f, n):
    """Patches whose closed (n+1)^3 node block holds a nonzero charge."""
    nz = f != 0
    ppa = (f.shape[0] - 1) // n
    return sum(bool(nz[a * n:a * n + n + 1, b * n:b * n + n + 1, c * n:c * n + n + 1].any())
               for a in range(ppa) for b in range(ppa) for c in range(ppa))


@pytest.mark.parametrize("conv", ["fp32", "fp64"])
@pytest.mark.parametrize("name", ["oscillatory_128", "smooth_128_l3", "sixth_64", "bumps_128_l3", "oscillatory_512_l4"])
def test_max_live_equals_skip_empty(name, conv):
    """A plan holding buffers for the live patches only (max_live = their
    count) gives the dense plan's phi element for element; one slot fewer is
    refused with MLC_ERR_OUT_OF_MEMORY."""
    import torch
    kw, charge = CASES[name]
    fh = charge()
    # a sixth-order plan's live patches are those of its modified right-hand side
    live = _live_count(sixth_order_rhs(fh) if kw.get("rhs_order") == 6 else fh, kw["n"])
    ppa = kw["N"] // kw["n"]
    print(f"{name} {conv}: {live} of {ppa ** 3} patches carry charge", flush=True)
    assert 0 < live < ppa ** 3 or name == "smooth_128_l3"
    f = torch.from_numpy(fh).cuda()
    dense = context().plan(gm.problem(conv=conv, skip_empty=1, **kw))
    a, _ = _solve(dense, f)
    dense.close()
    if live == ppa ** 3:
        live -= 1   # every patch is live: exercise the refusal only
    else:
        cap = context().plan(gm.problem(conv=conv, max_live=live, **kw))
        assert cap.info["slots"] == live
        b, _ = _solve(cap, f)
        assert torch.equal(a, b)
        cap.close()
    short = context().plan(gm.problem(conv=conv, max_live=live - 1, **kw))
    ws = torch.empty(short.workspace_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(gm.MLCError) as ei:
        short.solve(f, torch.empty_like(f), ws)
    assert ei.value.status == gm.MLC_ERR_OUT_OF_MEMORY and "max_live" in str(ei.value)
    short.close()


def test_max_live_reused_with_fewer_live_patches():
    """One max_live plan and workspace, two solves in a row: the second charge
    covers fewer patches, and each result equals the dense plan's."""
    import torch
    kw = dict(N=128, n=16, alpha=3.0, beta=6.0, P=4, Q=4, conv="fp32")
    f1 = mi.bump_charge(128, mi.bumps(3, 71, radius=(0.1, 0.15)))
    f2 = mi.bump_charge(128, mi.bumps(1, 72, radius=(0.08, 0.1)))
    n1, n2 = _live_count(f1, 16), _live_count(f2, 16)
    assert n2 < n1 < 512
    dense = context().plan(gm.problem(**kw))
    cap = context().plan(gm.problem(max_live=n1, **kw))
    ws = torch.empty(cap.workspace_bytes, dtype=torch.uint8, device="cuda")
    for fh in (f1, f2):
        f = torch.from_numpy(fh).cuda()
        a, _ = _solve(dense, f)
        b = torch.full_like(f, np.nan)
        cap.solve(f, b, ws)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
    dense.close()
    cap.close()


def test_max_live_analytic_and_refusals():
    """mlc_solve_analytic with a max_live plan equals the dense plan's; batches,
    graphs and the static scratch refuse such a plan."""
    import torch
    ctx = context()
    kw = dict(N=128, n=32, alpha=1.75, beta=3.25, P=4, Q=6, b=3, conv="fp64")
    dense = ctx.plan(gm.problem(**kw))
    cap = ctx.plan(gm.problem(max_live=40, **kw))
    out = []
    for plan in (dense, cap):
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        f = torch.empty((129,) * 3, dtype=torch.float64, device="cuda")
        phi = torch.full_like(f, np.nan)
        plan.solve_analytic(mi.oscillatory_terms(), 2, f, phi, ws)
        torch.cuda.synchronize()
        out.append(phi)
    assert torch.equal(out[0], out[1])
    f = torch.zeros((129,) * 3, dtype=torch.float64, device="cuda")
    ws = torch.empty(gm.batch_workspace_bytes([dense]), dtype=torch.uint8, device="cuda")
    with pytest.raises(gm.MLCError) as ei:
        gm.batch_workspace_bytes([dense, cap])
    assert ei.value.status == gm.MLC_ERR_UNSUPPORTED
    with pytest.raises(gm.MLCError) as ei:
        cap.solve_static(f, torch.empty_like(f))
    assert ei.value.status == gm.MLC_ERR_UNSUPPORTED
    dense.close()
    cap.close()


def test_max_live_box_domain():
    """A box domain with max_live: the live patches are found in the box's
    enclosing cube (f padded by zeros), and phi on the box equals the dense
    box solve's element for element."""
    import torch
    N, n = 96, 16
    fc = mi.bump_charge(N, mi.bumps(1, 91, radius=(0.08, 0.1), centre=(0.22, 0.28)))
    fb = np.ascontiguousarray(fc[:, :65, :49])
    assert np.array_equal(fc[:, 65:, :], np.zeros_like(fc[:, 65:, :])) and not fc[:, :, 49:].any()
    live = _live_count(fc, n)
    assert 0 < live < (N // n) ** 3
    kw = dict(N=(96, 64, 48), n=n, alpha=3.0, beta=6.0, P=4, Q=4, conv="fp64")
    f = torch.from_numpy(fb).cuda()
    dense = context().plan(gm.problem(skip_empty=1, **kw))
    cap = context().plan(gm.problem(max_live=live, **kw))
    a, _ = _solve(dense, f)
    b, _ = _solve(cap, f)
    assert torch.equal(a, b)
    dense.close()
    cap.close()
