"""Box domains (mlc_problem.box_cells) on MI355X: a B0 x B1 x B2-cell box is
solved inside its enclosing cube with f padded by zeros; the free-space
solution on the box does not depend on the padding.  Each box solve must
equal, element for element, the cube solve of the zero-padded charge
restricted to the box (two and three levels, float32 and float64, with and
without empty-patch skipping, alone and in a batch with a cube problem), and
approach the closed-form potential; MLC_CHECK checks the box's own faces."""
import numpy as np
import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

BUMPS = [mi.Bump((0.45, 0.35, 0.25), 0.2, 1.0), mi.Bump((0.6, 0.3, 0.3), 0.12, -0.5)]


def _box_fields(B, h):
    """Charge and closed-form potential on the box's nodes g h."""
    ax = [np.arange(b + 1) * h for b in B]
    X = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1).reshape(-1, 3)
    f = np.zeros(len(X))
    for bp in BUMPS:
        r = np.linalg.norm(X - np.asarray(bp.centre), axis=1) / bp.radius
        f += bp.weight * np.where(r < 1.0, (1.0 - r * r) ** 4, 0.0)
    phi = mi.bump_potential_at(X, BUMPS)
    shape = tuple(b + 1 for b in B)
    return f.reshape(shape), phi.reshape(shape)


CASES = [
    # (box cells, n, Q, levels, skip_empty)
    ((64, 48, 32), 16, 4, 2, 0),
    ((64, 48, 32), 16, 6, 2, 1),
    ((128, 64, 96), 16, 4, 3, 0),
]


@pytest.mark.parametrize("conv", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_box_equals_padded_cube(case, conv):
    import torch
    B, n, Q, levels, skip = CASES[case]
    h = 1.0 / max(B)
    ctx = context()
    pb = ctx.plan(gm.problem(tuple(B), n, 3.0, 6.0, 4, Q, conv=conv, levels=levels, skip_empty=skip,
                             origin=(0.0, 0.0, 0.0)))
    N = pb.info["N"]
    assert list(pb.info["box"]) == list(B) and N >= max(B) and N % n == 0
    fb, exact = _box_fields(B, h)
    fc = np.zeros((N + 1,) * 3)
    fc[:B[0] + 1, :B[1] + 1, :B[2] + 1] = fb
    pc = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, h=h, conv=conv, levels=levels, skip_empty=skip))
    out = []
    for plan, f in ((pb, fb), (pc, fc)):
        fd = torch.from_numpy(np.ascontiguousarray(f)).cuda()
        phi = torch.full_like(fd, np.nan)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.solve(fd, phi, ws)
        torch.cuda.synchronize()
        out.append(phi.cpu().numpy())
    box, cube = out
    err = float(np.abs(box - exact).max() / np.abs(exact).max())
    print(B, n, Q, levels, skip, conv, f"cube {N}, closed-form error {err:.2e}", flush=True)
    assert np.array_equal(box, cube[:B[0] + 1, :B[1] + 1, :B[2] + 1])
    assert err < 2e-3
    pb.close()
    pc.close()


def test_box_in_a_batch_and_checked(monkeypatch):
    import torch
    ctx = context()
    B = (64, 48, 32)
    h = 1.0 / 64
    pb = ctx.plan(gm.problem(B, 16, 3.0, 6.0, 4, 4, conv="fp32"))
    pc = ctx.plan(gm.problem(64, 16, 3.0, 6.0, 4, 4, conv="fp32"))
    fb = torch.from_numpy(_box_fields(B, h)[0]).cuda()
    fc = torch.from_numpy(mi.bump_charge(64, mi.bumps(2, 70, radius=(0.1, 0.2)))).cuda()
    alone = []
    for plan, f in ((pb, fb), (pc, fc)):
        phi = torch.empty_like(f)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
        plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        alone.append(phi)
    phis = [torch.full_like(fb, np.nan), torch.full_like(fc, np.nan)]
    ws = torch.empty(gm.batch_workspace_bytes([pb, pc]), dtype=torch.uint8, device="cuda")
    gm.solve_batched([pb, pc], [fb, fc], phis, ws)
    torch.cuda.synchronize()
    assert torch.equal(phis[0], alone[0]) and torch.equal(phis[1], alone[1])
    # the input check looks at the box's own faces
    monkeypatch.setenv("MLC_CHECK", "1")
    ws1 = torch.empty(pb.workspace_bytes, dtype=torch.uint8, device="cuda")
    phi = torch.empty_like(fb)
    pb.solve(fb, phi, ws1)
    for node in [(64, 10, 10), (10, 48, 10), (10, 10, 32), (0, 5, 5)]:
        bad = fb.clone()
        bad[node] = 1e-3
        with pytest.raises(gm.MLCError) as ei:
            pb.solve(bad, phi, ws1)
        assert ei.value.status == gm.MLC_ERR_INVALID_ARG, node
    torch.cuda.synchronize()
    pb.close()
    pc.close()
