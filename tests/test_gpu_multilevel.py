"""Multilevel MLC (paper sec. 5) on MI355X: a plan with levels = 3 or 4
solves the coarse charge by the method one level up, recursively.

Parity with the oracle's multilevel solve (oracle.mlc.mlc_solve_multilevel),
element by element: phi (float64 1e-12, float32 2e-6), and at the next
coarser level its node charge (F^H in the level box) and its uncorrected
solution.  Then the paper's three-level numbers for the smooth charge of
sec. 7.1 at N = 512 (27-point operator, 32^3-cell patches), and where this
implementation's three-level error comes from."""
import os

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import _slice, context, rel

pytestmark = pytest.mark.gpu

CASES = {
    # (N, n, alpha, beta, P, Q, levels, Z, inner radii of the coarser levels)
    "l3_64": (64, 8, 3.0, 6.0, 4, 6, 3, 64, ()),
    "l3_128": (128, 16, 3.0, 6.0, 4, 6, 3, 128, ()),
    "l4_128": (128, 8, 3.0, 6.0, 4, 4, 4, 64, ()),
    # a larger alpha at the coarser levels (sec. 7.2)
    "l3_64_alpha": (64, 8, 2.0, 3.0, 4, 6, 3, 64, (3.0,)),
    "l4_128_alpha": (128, 8, 2.0, 4.0, 5, 4, 4, 64, (3.0, 2.0)),
}


def _gpu(name, conv):
    import torch
    N, n, a, b, P, Q, levels, Z, la = CASES[name]
    f = mi.smooth_charge(N)
    plan = context().plan(gm.problem(N, n, a, b, P, Q, conv=conv, Z=Z, levels=levels, level_alpha=la))
    fd = torch.from_numpy(f).cuda()
    phi = torch.empty_like(fd)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve(fd, phi, ws)
    torch.cuda.synchronize()
    E = plan.info["level_N"] + 1
    out = dict(f=f, phi=phi.cpu().numpy(), info=plan.info,
               lf=_slice(ws, plan, gm.MLC_VIEW_LEVEL_CHARGE, torch.float64, (E, E, E)),
               lphi=_slice(ws, plan, gm.MLC_VIEW_LEVEL_PHI, torch.float64, (E, E, E)))
    plan.close()
    return out


@pytest.mark.parametrize("name", sorted(CASES))
def test_multilevel_fp64_parity(name):
    N, n, a, b, P, Q, levels, Z, la = CASES[name]
    g = _gpu(name, "fp64")
    prm = omlc.Params(N=N, n=n, alpha=a, beta=b, P=P, Q=Q, Z=Z)
    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        phi, trail = omlc.mlc_solve_multilevel(g["f"], prm, levels, dgf_cached(Q, Z), level_alpha=la)
    assert g["info"]["level_alpha"][:len(la)] == list(la)
    assert g["info"]["level_margin"] == omlc.level_box_margin(prm, deeper=levels > 3)
    errs = {"phi": rel(g["phi"], phi), "level_charge": rel(g["lf"], trail[1][3]),
            "level_phi": rel(g["lphi"], trail[1][0])}
    ex = mi.smooth_potential(N)
    print(name, {k: f"{v:.2e}" for k, v in errs.items()},
          f"closed-form error {np.abs(g['phi'] - ex).max() / np.abs(ex).max():.3e}", flush=True)
    for k, v in errs.items():
        assert v < 1e-12, (k, v)


def test_multilevel_fp32_close_to_fp64():
    a = _gpu("l3_128", "fp64")
    b = _gpu("l3_128", "fp32")
    assert rel(b["phi"], a["phi"]) < 2e-6


# three-level errors of the smooth charge at N = 512 printed in the paper
# (sec. 7.1, the three-level tables; finest level)
PAPER_512 = {
    # (alpha, beta, P): error
    (2.0, 2.0, 1): 1.30594e-7,
    (1.75, 3.25, 1): 5.26000e-7,
    (1.75, 3.25, 4): 1.0782e-6,
    (1.75, 3.25, 6): 1.1101e-6,
    (1.75, 3.25, 8): 1.4926e-7,
}


def _solve_smooth(N, a, b, P, levels, level_alpha=()):
    import torch
    f = torch.from_numpy(mi.smooth_charge(N)).cuda()
    phi = torch.empty_like(f)
    plan = context().plan(gm.problem(N, 32, a, b, P, 6, conv="fp64", levels=levels, level_alpha=level_alpha))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve(f, phi, ws)
    torch.cuda.synchronize()
    out = phi.cpu().numpy()
    lphi = None
    if levels > 2:
        E = plan.info["level_N"] + 1
        m = plan.info["level_margin"]
        w = N // 4 + 1
        lphi = _slice(ws, plan, gm.MLC_VIEW_LEVEL_PHI, torch.float64, (E, E, E))[m:m + w, m:m + w, m:m + w]
    del ws, f, phi
    plan.close()
    torch.cuda.empty_cache()
    return out, lphi


def test_three_level_smooth_512():
    """The three-level errors at N = 512 against the paper's, and where ours
    come from.  In this implementation the level-1 solve is the two-level
    method applied to the level charge F^H on the grid of spacing 4h, and
    its error against the exact discrete solution G^{4h} * F^H is what the
    two-level method makes on the charge itself at N = 128: the three-level
    error at N = 512 equals the two-level error against the discrete
    solution at N = 128 (to 25 %, the finest level's own error adds to it).
    That identity is asserted; so are the paper's findings that hold here:
    MLC-0 with a wide radius keeps the two-level error (alpha = beta = 3,
    the widest built, at N = 256; against the paper's beta = 3.25 whose 4.86e-9 needs a
    local torus above the built sizes), every level's solution carries the
    finest level's error (the level-1 solution, corrected by C2 h^2 f with
    the finest spacing, is within a factor 2 of the finest level's), and
    the MLC runs (alpha = 1.75) lose more than a factor 20 against that
    MLC-0 (the paper's smallest such loss is 30, at P = 8).  The remaining
    values differ from the paper's by factors of 2 to 30 and are printed."""
    from oracle import convolution as oconv
    N = 512
    ex = mi.smooth_potential(N)
    scale = np.abs(ex).max()
    ex1 = mi.smooth_potential(N // 4)
    corr1 = mi.smooth_charge(N // 4) / (12.0 * N * N)
    # the exact discrete solution at N = 128, corrected
    N2 = N // 4
    f2 = mi.smooth_charge(N2)
    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        disc = oconv.conv_hockney(dgf_cached(6, 128), 128, f2, np.zeros(3, int), np.full(3, N2),
                                  M=2 * N2 + 1) / N2 ** 2 + f2 / (12.0 * N2 * N2)
    got = {}
    for (a, b, P), paper in PAPER_512.items():
        phi, lphi = _solve_smooth(N, a, b, P, 3)
        e3 = float(np.abs(phi - ex).max() / scale)
        e1 = float(np.abs(lphi + corr1 - ex1).max() / scale)
        phi2, _ = _solve_smooth(N2, a, b, P, 2)
        e2 = float(np.abs(phi2 - disc).max() / np.abs(disc).max())
        got[(a, b, P)] = e3
        print(f"3 levels N 512 alpha {a} beta {b} P {P}: finest {e3:.3e}, level 1 {e1:.3e} "
              f"(paper {paper:.3e}); two levels at N 128 against the discrete solution {e2:.3e}", flush=True)
        assert abs(e3 - e2) < 0.25 * e2, (a, b, P, e3, e2)
        assert e1 < 2 * e3 and e3 < 2 * e1, (a, b, P, e1, e3)
    # MLC-0 with the widest built radius: the number of levels does not
    # change its error (at N = 256, where the two-level coarse grid fits the
    # built transform sizes), and at N = 512 it stays far below the MLC runs
    w = {}
    for n_, lv in ((256, 2), (256, 3), (512, 3)):
        phi, _ = _solve_smooth(n_, 3.0, 3.0, 1, lv)
        ex_ = ex if n_ == N else mi.smooth_potential(n_)
        w[(n_, lv)] = float(np.abs(phi - ex_).max() / np.abs(ex_).max())
    print("MLC-0 alpha = beta = 3:", {k: f"{v:.3e}" for k, v in w.items()}, flush=True)
    assert w[(256, 3)] < 2 * w[(256, 2)]
    for P in (1, 4, 6, 8):
        assert got[(1.75, 3.25, P)] > 20 * w[(512, 3)]


# two-level errors of the smooth charge at N = 512 with alpha = 1.75,
# beta = 3.25 (the paper's Table 7); the two-level coarse grid of that case
# is above the built transform sizes, three levels reach it
PAPER_T7_512 = {1: 5.42412e-8, 4: 9.16574e-9, 6: 5.99534e-9, 9: 6.02843e-9}


def test_coarse_alpha_recovers_two_level_errors_512():
    """Sec. 7.2's remedy: a larger inner radius at the coarser level only
    (alpha = 3 there, 1.75 at the finest level, beta = 3.25) brings the
    three-level errors at N = 512 to the paper's two-level ones for the same
    finest-level parameters (Table 7): no more than 1.5 times the paper's and
    no less than half of it for P = 1, 4, 6, 9 (at P = 6 and 9 ours are 0.73
    and 0.66 of the paper's), where the same radius at both levels is 10 to
    1000 times worse."""
    N = 512
    ex = mi.smooth_potential(N)
    scale = np.abs(ex).max()
    for P, paper in PAPER_T7_512.items():
        wide, _ = _solve_smooth(N, 1.75, 3.25, P, 3, (3.0,))
        e = float(np.abs(wide - ex).max() / scale)
        print(f"3 levels N 512 alpha 1.75 (3 at level 1) beta 3.25 P {P}: {e:.3e} (paper, two levels: {paper:.3e})",
              flush=True)
        assert paper / 2 < e < 1.5 * paper, (P, e, paper)
