"""The paper's own four-level runs of the oscillatory charges at N = 2048
(sec. 7.2, Tables 12 and 14: L27, beta = 3.25, 32^3-cell patches, P = 1) on
one GPU, the plan keeping per-patch convolution buffers for the live patches
only (max_live).  The scaled maximum error of the finest level over all
2049^3 nodes, against the closed-form potential, is compared with the value
the paper prints: within 15 % (measured 6-8 % above), and the raised coarse
radii of Table 14 more than halve Table 12's error, as printed.  Skipped when
the device lacks the 245 GiB the arrays and the workspace take."""
import gc

import pytest

import mlc_inputs as mi
from paper_1702_08111_amd import mlc as gm

from gpu_common import context

pytestmark = pytest.mark.gpu

N, n = 2048, 32
# (coarser-level radii from the finest level up, the paper's error at l = 3, P = 1)
SETTINGS = {"table_14": ((2.0, 2.25), 1.22595e-6), "table_12": ((1.75, 1.75), 2.74856e-6)}


def _scaled_error(phi, dev):
    """max |phi - closed form| / max |closed form| over every node, in slabs
    (nan if phi holds a non-finite value)."""
    import torch
    ax = torch.arange(N + 1, dtype=torch.float64, device=dev) / N
    err = scale = 0.0
    for k0 in range(0, N + 1, 8):
        k1 = min(k0 + 8, N + 1)
        exact = torch.zeros((k1 - k0, N + 1, N + 1), dtype=torch.float64, device=dev)
        for c in mi.OSC_CENTRES:
            r = torch.sqrt(((ax[k0:k1] - c[0]) ** 2)[:, None, None] + ((ax - c[1]) ** 2)[None, :, None]
                           + ((ax - c[2]) ** 2)[None, None, :]) / mi.OSC_RO
            exact += mi._osc_psi(r, xp=torch) / mi.OSC_RO
            del r
        d = (phi[k0:k1] - exact).abs()
        if not bool(torch.isfinite(d).all()):
            return float("nan")
        err = max(err, float(d.max()))
        del d
        scale = max(scale, float(exact.abs().max()))
        del exact
    return err / scale


def test_oscillatory_2048_four_levels_matches_tables_12_and_14():
    import torch
    dev = torch.device("cuda:0")
    probs = {t: gm.problem(N, n, 1.75, 3.25, 1, 6, conv="fp64", levels=4, level_alpha=la, max_live=1024)
             for t, (la, _) in SETTINGS.items()}
    ws_bytes = max(gm.problem_workspace_bytes(p) for p in probs.values())
    node_bytes = 8 * (N + 1) ** 3
    gc.collect()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    if free < ws_bytes + 2 * node_bytes + (8 << 30):
        pytest.skip(f"needs {(ws_bytes + 2 * node_bytes) / 2 ** 30:.0f} GiB of device memory, {free / 2 ** 30:.0f} free")
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    f = torch.empty((N + 1,) * 3, dtype=torch.float64, device=dev)
    phi = torch.empty_like(f)
    errs = {}
    try:
        for table, prob in probs.items():
            plan = context().plan(prob)
            # the library samples the radial terms into f, then a plain solve of that f
            plan.solve_analytic(mi.oscillatory_terms(), 2, f, phi, ws)
            phi.fill_(float("nan"))
            plan.solve(f, phi, ws)
            torch.cuda.synchronize()
            plan.close()
            errs[table] = _scaled_error(phi, dev)
            paper = SETTINGS[table][1]
            print(f"2048^3 {table} P=1: error {errs[table]:.5e}, paper {paper:.5e}", flush=True)
            assert 0.85 < errs[table] / paper < 1.15
        assert errs["table_12"] > 2.0 * errs["table_14"]
    finally:
        del ws, f, phi
        gc.collect()
        torch.cuda.empty_cache()
