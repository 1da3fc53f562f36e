"""Charges given analytically (mlc_solve_analytic) on MI355X: the library
samples the radial terms on the nodes and takes each patch's Legendre
coefficients by composite Gauss integration (paper sec. 4.1 step 1).

Checked against the oracle solving the same problem with the same Gauss
coefficients (oracle.legendre.moments_gauss of the terms as given by
mlc_inputs): the sampled charge to rounding, phi within 1e-12 (float64
convolutions) and 2e-6 (float32), the coefficients within 1e-12; the Gauss
coefficients differ from the Boole ones of the same node values (the path is
really taken); a term reaching the outer boundary is refused."""
import os

import numpy as np
import pytest
import scipy.fft

import mlc_inputs as mi
from oracle import legendre as leg
from oracle import mlc as omlc
from oracle.dgf import dgf_cached
from paper_1702_08111_amd import mlc as gm

from gpu_common import _slice, context, oracle_params, rel

pytestmark = pytest.mark.gpu

CASES = {
    # (N, n, Q, terms, gauss points, Z)
    "bumps_64": (64, 16, 4, lambda: mi.bump_terms(mi.bumps(3, 91, radius=(0.12, 0.2))), 4, 128),
    "smooth_64": (64, 16, 6, mi.smooth_terms, 3, 128),
    "oscillatory_128": (128, 32, 6, mi.oscillatory_terms, 4, 128),
    "bumps_32_p9": (32, 8, 4, lambda: mi.bump_terms(mi.bumps(2, 92, radius=(0.15, 0.25))), 2, 64),
}
P_OF = {"bumps_32_p9": 9}


def _run(name, conv):
    import torch
    N, n, Q, terms_fn, g, Z = CASES[name]
    terms = terms_fn()
    P = P_OF.get(name, 4)
    plan = context().plan(gm.problem(N, n, 3.0, 6.0, P, Q, conv=conv, Z=Z))
    f = torch.full(((N + 1),) * 3, float("nan"), dtype=torch.float64, device="cuda")
    phi = torch.empty_like(f)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve_analytic(terms, g, f, phi, ws)
    torch.cuda.synchronize()
    mom = _slice(ws, plan, gm.MLC_VIEW_MOMENTS, torch.float64, (plan.info["npatch"], plan.info["K"]))
    out = dict(f=f.cpu().numpy(), phi=phi.cpu().numpy(), moments=mom, info=plan.info)
    # the same node values through the Boole path
    phi_b = torch.empty_like(f)
    plan.solve(f, phi_b, ws)
    torch.cuda.synchronize()
    out["moments_boole"] = _slice(ws, plan, gm.MLC_VIEW_MOMENTS, torch.float64, (plan.info["npatch"], plan.info["K"]))
    plan.close()
    return terms, g, out


@pytest.mark.parametrize("name", sorted(CASES))
def test_analytic_fp64_parity(name):
    terms, g, out = _run(name, "fp64")
    info = out["info"]
    N, n = info["N"], info["n"]
    fn = mi.radial_charge_nodes(N, terms)
    assert rel(out["f"], fn) < 1e-14
    prm = oracle_params(info, 3.0, 6.0)
    h, R = prm.hh, prm.R

    def gauss(i):
        corner = n * np.asarray(i) * h
        return leg.moments_gauss(lambda a, b, c: mi.radial_charge_at(a, b, c, terms), corner, n, h, prm.P, R, g)

    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        phi, o = omlc.mlc_solve(fn, prm, dgf_cached(prm.Q, prm.Z), keep=True, moments_fn=gauss)
    em, ep = rel(out["moments"], o["moments"]), rel(out["phi"], phi)
    eb = rel(out["moments"], out["moments_boole"])
    print(name, f"moments {em:.2e}, phi {ep:.2e}, Gauss vs Boole moments {eb:.2e}", flush=True)
    assert em < 1e-12 and ep < 1e-12
    assert eb > 1e-12


@pytest.mark.parametrize("name", ["bumps_64", "oscillatory_128"])
def test_analytic_fp32_close_to_fp64(name):
    _, _, a = _run(name, "fp64")
    _, _, b = _run(name, "fp32")
    assert np.array_equal(a["f"], b["f"])
    assert rel(b["moments"], a["moments"]) < 1e-12
    assert rel(b["phi"], a["phi"]) < 2e-6


def test_analytic_refuses_a_charge_on_the_boundary():
    import torch
    plan = context().plan(gm.problem(32, 8, 3.0, 6.0, 4, 4, conv="fp64", Z=64))
    f = torch.zeros((33,) * 3, dtype=torch.float64, device="cuda")
    phi = torch.empty_like(f)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(gm.MLCError) as ei:
        plan.solve_analytic([((0.1, 0.5, 0.5), 0.2, 1.0, 0.0, gm.MLC_PROFILE_BUMP)], 4, f, phi, ws)
    assert ei.value.status == gm.MLC_ERR_INVALID_ARG
    plan.close()


def test_analytic_multilevel_parity():
    """A charge given analytically on a three-level plan: the finest level's
    coefficients by Gauss integration, the coarser level from its node
    charge; against the oracle's multilevel solve with the same Gauss
    coefficients at the finest level."""
    import torch
    N, n, Q, Z, g = 64, 8, 6, 64, 3
    terms = mi.smooth_terms()
    plan = context().plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp64", Z=Z, levels=3))
    f = torch.full(((N + 1),) * 3, float("nan"), dtype=torch.float64, device="cuda")
    phi = torch.empty_like(f)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    plan.solve_analytic(terms, g, f, phi, ws)
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    plan.close()
    prm = omlc.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=Q, Z=Z)
    h, R = prm.hh, prm.R

    def gauss(i):
        corner = n * np.asarray(i) * h
        return leg.moments_gauss(lambda a, b, c: mi.radial_charge_at(a, b, c, terms), corner, n, h, prm.P, R, g)

    with scipy.fft.set_workers(len(os.sched_getaffinity(0))):
        ref, _ = omlc.mlc_solve_multilevel(mi.radial_charge_nodes(N, terms), prm, 3, dgf_cached(Q, Z),
                                           moments_fn=gauss)
    e = rel(got, ref)
    print(f"analytic charge, three levels: {e:.2e}", flush=True)
    assert e < 1e-12
