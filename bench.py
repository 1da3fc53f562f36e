"""Benchmark of the two-level MLC solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload fp32_256_q6]

One step = one full two-level MLC solve (local convolutions, moments, coarse
right-hand side, coarse solve, skeleton boundary values, Dirichlet solves,
correction) of a 256^3 problem whose charge already sits in HBM.  Prints one
JSON line: grid points/s (N^3 per solve) of the float32-convolution path,
with the float64 path, the errors, p50/p99 latency, the roofline of the
dominant kernel and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

import mlc_inputs as mi

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # MI355X fp32 vector
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="fp32_256_q6")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--batch-steps", type=int, default=5,
                    help="timed steps of the 64-problem uneven batch (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="measured requests of the serving loop after 50 warm-ups (0: skip)")
    ap.add_argument("--serve-load", type=float, default=0.7, help="arrival rate / saturation rate")
    ap.add_argument("--no-sweep", action="store_true", help="skip the (alpha, beta, P, Q) sweep")
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the headline workload's solves with empty patches skipped (profiles of the dense "
                         "kernels then see dense launches only)")
    ap.add_argument("--ml-steps", type=int, default=3,
                    help="timed solves per multilevel workload (512^3 three levels, 1024^3 four levels); 0 skips")
    ap.add_argument("--osc-steps", type=int, default=5,
                    help="timed steps of the oscillatory 384^3 workload per path (0: skip)")
    ap.add_argument("--paper-2048", action="store_true",
                    help="instead of the headline line: the oscillatory charges of sec. 7.2 at 2048^3 with four "
                         "levels, Tables 12 and 14's settings (P = 1 and 4), errors over every node")
    return ap.parse_args()


def kernel_model(info):
    """Algorithmic bytes and flops per launch of each local-convolution kernel
    (whole batch of patches), split from the whole-solve model below: per
    patch, the forward intermediate (n+1)^2 (M/2+1) complex values and the
    output-side one W^2 (M/2+1), W = n + 2 d_alpha + 8b + 1 the local field
    box, each written once and read once, plus the patch charge in and the
    coarse samples and skeleton planes out:
      conv_xdft  (n+1)^3 8 (f) + (n+1)^2 (M/2+1) c
      conv_yz    (n+1)^2 (M/2+1) c + W^2 (M/2+1) c + the DGF spectrum once
      conv_out   W^2 (M/2+1) c + (Wc^3 + 3 planes Wa^2) o
    (c = complex, o = real conv-precision bytes).  Flops: nominal FFT counts
    5 L log2 L per complex line of length L, 4 per real x complex MAC,
    2 per real x complex product."""
    conv = 4 if info["conv_precision"] == 1 else 8       # bytes per real in conv precision
    cb = 2 * conv                                        # complex
    n, M, P = info["n"], info["M"], info["npatch"]
    S, Mh = n + 1, M // 2 + 1
    W = n + 2 * info["d_alpha"] + 8 * info["b"] + 1
    Wp = info["Wa"] + 2 * info["b"]
    Wc, Wa, npl = info["Wc"], info["Wa"], info["nplanes_a"]
    lg = np.log2(M)
    fft = 5.0 * M * lg
    X = P * Mh * S * S * cb
    Zw = P * W * W * Mh * cb
    outs = P * (Wc ** 3 + 3 * npl * Wa * Wa) * conv
    return {
        "conv_xdft": dict(bytes=P * S ** 3 * 8 + X, flops=P * S * Mh * S * S * 4.0),
        "conv_yz": dict(bytes=X + Zw + Mh ** 3 * conv,
                        flops=P * Mh * (S * fft + M * 2 * fft + 2.0 * M * M)),
        "conv_out": dict(bytes=Zw + outs, flops=P * Wp * (Mh * fft + ((Wp + 1) // 2) * fft)),
    }


def solve_model(info):
    """Whole-solve model of the path (independent of how the kernels are
    split): compulsory HBM bytes if each patch's two pruned spectral
    intermediates make one round trip, and nominal FFT flops.
      bytes = patches x [2((n+1)^2 + W^2)(M/2+1) c + (coarse samples + planes) o]
              + 3 (N+1)^3 8 + 5 M_c^3 16 (the coarse torus: fill and pruned passes)
      flops = patches x [(n+1)^2 F_r + (n+1)(M/2+1) F_c + M(M/2+1) F_c   (forward)
                         + 2 M^2 (M/2+1)                                  (DGF multiply)
                         + M(M/2+1) F_c + W(M/2+1) F_c + W^2 F_r]         (inverse)
    with W = n + 2 d_alpha + 8b + 1 the local field box, F_c = 5 M log2 M per
    complex line and F_r = F_c / 2 per real line."""
    conv = 4 if info["conv_precision"] == 1 else 8
    c = 2 * conv
    n, M, P, N = info["n"], info["M"], info["npatch"], info["N"]
    W = n + 2 * info["d_alpha"] + 8 * info["b"] + 1
    Mh = M // 2 + 1
    outs = info["Wc"] ** 3 + 3 * info["nplanes_a"] * info["Wa"] ** 2
    nbytes = P * (2 * ((n + 1) ** 2 + W ** 2) * Mh * c + outs * conv) + 3 * (N + 1) ** 3 * 8 \
        + 5 * info["M_coarse"] ** 3 * 16
    Fc = 5.0 * M * np.log2(M)
    Fr = Fc / 2
    flops = P * ((n + 1) ** 2 * Fr + (n + 1) * Mh * Fc + M * Mh * Fc + 2.0 * M * M * Mh
                 + M * Mh * Fc + W * Mh * Fc + W * W * Fr)
    return nbytes, flops


KERNEL_SOURCES = ["paper_1702_08111_amd/csrc/conv_kernels.h", "paper_1702_08111_amd/csrc/fft_reg.h",
                  "paper_1702_08111_amd/csrc/fft.h", "paper_1702_08111_amd/csrc/common.h"]


def kernel_source_hash():
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE x its copy-kernel scale + WRITE_SIZE), or None when no
    summary exists or the kernel sources changed since it was taken."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for ln in open(path):
        if "=" in ln and ln.strip().startswith("- `"):
            k, v = ln.strip()[3:].split("`", 1)[0].split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != kernel_source_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(name):
    """The oracle (oracle/, float64 NumPy/SciPy, untuned, SciPy FFTs with one
    worker per available core) solving the same workload once, timed.  The
    DGF table and the Legendre far-field tables are plan-time work (built
    before a solve on the GPU too) and stay outside the timed region.
    Returns the baseline record and the oracle's phi, against which the GPU
    solves' errors are stated."""
    import scipy.fft
    from oracle import mlc as om
    from oracle.dgf import dgf

    cores = len(os.sched_getaffinity(0))
    N, n, Q, bumps = mi.workload(name)
    f = mi.bump_charge(N, bumps)
    prm = om.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=Q, Z=128)
    with scipy.fft.set_workers(cores):
        progress("CPU oracle: DGF table (plan time, not timed)")
        G1 = dgf(Q, 128)
        progress("CPU oracle: far-field tables (plan time, not timed)")
        tables = om.plan_tables(G1, prm)
        progress("CPU oracle: one full two-level solve (timed)")
        t0 = time.perf_counter()
        phi = om.mlc_solve(f, prm, G1, tables=tables)
        t = time.perf_counter() - t0
    rec = {"value": float(N ** 3 / t), "unit": "grid points/s", "cores": cores, "kind": "oracle",
           "sample": (f"one full oracle solve of this workload ({N}^3, {(N // n) ** 3} patches): step-1 local "
                      f"fields, moments, coarse right-hand side, coarse solve, boundary values, Dirichlet solves "
                      f"and correction in {t:.1f} s; DGF and far-field tables built beforehand, not timed")}
    return rec, phi


def cpu_baseline_direct(sample_patches=8):
    """The oracle with its local convolutions as literal sums (mode direct),
    single process: the full 32^3 solve, and the step-1 local fields of a
    sample of the 128^3 workload's patches scaled to all of them (the whole
    128^3 direct solve would take minutes).  Plan-time tables are built by
    FFT beforehand and not timed."""
    from oracle import mlc as om
    from oracle.dgf import dgf_cached
    out = {"kind": "oracle", "mode": "direct", "cores": 1}
    N, n, Q, bumps = mi.workload("fp64_32")
    f = mi.bump_charge(N, bumps)
    prm = om.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=Q, Z=64)
    G1 = dgf_cached(Q, 64)
    tables = om.plan_tables(G1, prm)
    t0 = time.perf_counter()
    om.mlc_solve(f, prm, G1, conv_mode="direct", tables=tables)
    t = time.perf_counter() - t0
    out["fp64_32"] = {"value": float(N ** 3 / t), "unit": "grid points/s",
                      "sample": f"one full solve of the 32^3 workload ({(N // n) ** 3} patches) in {t:.2f} s"}
    N, n, Q, bumps = mi.workload("fp32_128")
    f = mi.bump_charge(N, bumps)
    prm = om.Params(N=N, n=n, alpha=3.0, beta=6.0, P=4, Q=Q, Z=128)
    G1 = dgf_cached(Q, 128)
    patches = om.patch_indices(N, n)
    pick = patches[np.linspace(0, len(patches) - 1, sample_patches).astype(int)]
    t0 = time.perf_counter()
    for i in pick:
        om.local_field(G1, prm, om.patch_charge(f, n, i), mode="direct")
    t = (time.perf_counter() - t0) * len(patches) / len(pick)
    out["fp32_128_local_fields"] = {
        "value": float(N ** 3 / t), "unit": "grid points/s",
        "sample": f"step-1 local fields of {len(pick)} of the {len(patches)} patches of the 128^3 workload by "
                  f"literal sums, scaled to all patches ({t:.0f} s); the other steps not included"}
    return out


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def batch_bench(ctx, steps, dev):
    """The 64-problem uneven batch (N in {32, 64, 96, 128, 192}, 16^3-cell
    patches, L19, float32 convolutions, 1-4 seeded bumps each) solved by
    one mlc_solve_batched call per step."""
    import torch
    from paper_1702_08111_amd import mlc as gm
    probs = mi.batch_problems()
    plans_by_n = {}
    plans = []
    for N, _ in probs:
        if N not in plans_by_n:
            plans_by_n[N] = ctx.plan(gm.problem(N, 16, 3.0, 6.0, 4, 4, conv="fp32", fft_size=-1))
        plans.append(plans_by_n[N])
    fs = [torch.from_numpy(mi.bump_charge(N, b)).to(dev) for N, b in probs]
    phis = [torch.empty_like(f) for f in fs]
    ws = torch.empty(gm.batch_workspace_bytes(plans), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    gm.solve_batched(plans, fs, phis, ws, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        gm.solve_batched(plans, fs, phis, ws, stream)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    points = sum(N ** 3 for N, _ in probs)
    # the same batch captured once by the library and replayed as one graph
    g = gm.BatchGraph(plans, fs, phis, ws)
    g.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch(stream)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / steps
    g.close()
    out = {"value": points / (ms * 1e-3), "unit": "grid points/s", "ms_per_step": ms,
           "graph_ms_per_step": gms, "graph_value": points / (gms * 1e-3),
           "out_planes_autotuned": plans[0].info["out_planes"],
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "problems": len(probs), "patches": int(sum(p.info["npatch"] for p in plans)),
           "workspace_gb": round(ws.numel() / 1e9, 2), "fft_size_autotuned": plans[0].info["M"],
           "config": "64 problems, N ~ U{32,64,96,128,192} (seed 104), 16^3-cell patches, L19, P=4, "
                     "alpha=3, beta=6, fp32 convolutions, autotuned local torus, one mlc_solve_batched call"}
    del ws, fs, phis
    for p in plans_by_n.values():
        p.close()
    torch.cuda.empty_cache()
    return out


def oscillatory_bench(ctx, steps, dev, N=384, n=32, Q=6):
    """The oscillatory three-charge workload of sec. 7.2 (gamma = 28 pi,
    Ro = 1/20) at the largest convenient two-level size (384^3, 32^3-cell
    patches, L27): float32 and float64 solves timed, errors against the
    closed form and between the two paths."""
    import torch
    from paper_1702_08111_amd import mlc as gm
    f = torch.from_numpy(mi.oscillatory_charge(N)).to(dev)
    exact = mi.oscillatory_potential(N)
    out = {"config": f"oscillatory three-charge charge (sec. 7.2), {N}^3, {n}^3-cell patches "
                     f"({(N // n) ** 3}), L27, alpha=3, beta=6, P=4"}
    phis = {}
    for conv in ("fp32", "fp64"):
        plan = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv))
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        phi = torch.empty_like(f)
        plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        phis[conv] = phi.cpu().numpy()
        out[conv] = {"ms_per_step": ms, "value": N ** 3 / (ms * 1e-3), "unit": "grid points/s",
                     "vs_closed_form": float(np.abs(phis[conv] - exact).max() / np.abs(exact).max())}
        del ws
        plan.close()
    out["fp32_vs_fp64_relmax"] = float(np.abs(phis["fp32"] - phis["fp64"]).max() / np.abs(phis["fp64"]).max())
    torch.cuda.empty_cache()
    return out


def multilevel_bench(ctx, steps, dev):
    """The multilevel method (sec. 5): the smooth charge of sec. 7.1 at 512^3
    with three levels (alpha = 1.75 at the finest level and 3 at the next,
    sec. 7.2's remedy; beta = 3.25, P = 4, L27), float64 and float32 local
    convolutions, errors against the closed form; and the oscillatory
    charges of sec. 7.2 at 1024^3 with four levels (alpha = 1.75, 2, 2.25
    from the finest level up), float32 convolutions, the charge sampled on the
    device from its radial terms, the error taken on every fourth node."""
    import torch
    from paper_1702_08111_amd import mlc as gm

    def timed(plan, f, phi, ws):
        plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    out = {}
    N = 512
    f = torch.from_numpy(mi.smooth_charge(N)).to(dev)
    exact = mi.smooth_potential(N)
    scale = np.abs(exact).max()
    rows = {}
    for conv in ("fp64", "fp32"):
        plan = ctx.plan(gm.problem(N, 32, 1.75, 3.25, 4, 6, conv=conv, levels=3, level_alpha=(3.0,)))
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        phi = torch.empty_like(f)
        ms = timed(plan, f, phi, ws)
        rows[conv] = {"ms_per_step": ms, "value": N ** 3 / (ms * 1e-3), "unit": "grid points/s",
                      "vs_closed_form": float(np.abs(phi.cpu().numpy() - exact).max() / scale),
                      "workspace_GiB": plan.workspace_bytes / 2 ** 30}
        del ws, phi
        plan.close()
        torch.cuda.empty_cache()
    out["smooth_512_three_levels"] = {
        "config": "smooth charge (sec. 7.1), 512^3, 32^3-cell patches, L27, 3 levels, alpha 1.75 (3 at level 1), "
                  "beta 3.25, P 4; the paper's two-level error for these finest-level parameters (Table 7) "
                  "is 9.17e-9", **rows}
    del f
    torch.cuda.empty_cache()
    progress("multilevel: oscillatory workload, 1024^3, four levels")
    N, stride = 1024, 4
    plan = ctx.plan(gm.problem(N, 32, 1.75, 3.25, 4, 6, conv="fp32", levels=4, level_alpha=(2.0, 2.25)))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    f = torch.empty((N + 1,) * 3, dtype=torch.float64, device=dev)
    phi = torch.empty_like(f)
    # the library samples the radial terms into f (the solve it runs here is a warmup)
    plan.solve_analytic(mi.oscillatory_terms(), 2, f, phi, ws)
    ms = timed(plan, f, phi, ws)
    got = phi[::stride, ::stride, ::stride].cpu().numpy()
    # the same solve with empty patches skipped (most of this grid has no charge)
    sp = ctx.plan(gm.problem(N, 32, 1.75, 3.25, 4, 6, conv="fp32", levels=4, level_alpha=(2.0, 2.25), skip_empty=1))
    phs = torch.empty_like(f)
    ms_sparse = timed(sp, f, phs, ws)
    same = bool(torch.equal(phs, phi))
    del phs
    sp.close()
    ax = np.arange(0, N + 1, stride) / N
    exact = np.zeros(got.shape)
    for c in mi.OSC_CENTRES:
        r = np.sqrt((ax[:, None, None] - c[0]) ** 2 + (ax[None, :, None] - c[1]) ** 2
                    + (ax[None, None, :] - c[2]) ** 2) / mi.OSC_RO
        exact += mi._osc_psi(r) / mi.OSC_RO
    out["oscillatory_1024_four_levels"] = {
        "config": "oscillatory charges (sec. 7.2), 1024^3, 32^3-cell patches, L27, 4 levels, alpha 1.75 / 2 / 2.25 "
                  "from the finest level up, beta 3.25, P 4, float32 local convolutions; error on every 4th node",
        "ms_per_step": ms, "value": N ** 3 / (ms * 1e-3), "unit": "grid points/s",
        "vs_closed_form_sampled": float(np.abs(got - exact).max() / np.abs(exact).max()),
        "workspace_GiB": plan.workspace_bytes / 2 ** 30,
        "empty_patches_skipped": {"ms_per_step": ms_sparse, "value": N ** 3 / (ms_sparse * 1e-3),
                                  "equal_to_dense": same}}
    del ws, f, phi
    plan.close()
    torch.cuda.empty_cache()
    return out


def _osc_live_patches(N, n):
    """Patches of an N^3 grid of n^3-cell patches holding a node strictly inside
    one of the oscillatory charges' balls (other than its centre): the
    patches with charge."""
    ppa = N // n
    live = np.zeros((ppa,) * 3, dtype=bool)
    for c in mi.OSC_CENTRES:
        lo = [max(int(np.floor((c[d] - mi.OSC_RO) * N)), 0) for d in range(3)]
        hi = [min(int(np.ceil((c[d] + mi.OSC_RO) * N)), N) for d in range(3)]
        ax = [np.arange(lo[d], hi[d] + 1) for d in range(3)]
        r = np.sqrt(((ax[0] / N - c[0]) ** 2)[:, None, None] + ((ax[1] / N - c[1]) ** 2)[None, :, None]
                    + ((ax[2] / N - c[2]) ** 2)[None, None, :]) / mi.OSC_RO
        idx = np.argwhere((r < 1.0) & (r > 0.0)) + np.asarray(lo)
        # a node on a patch face belongs to the patches on both sides
        for s0 in (0, 1):
            for s1 in (0, 1):
                for s2 in (0, 1):
                    q = (idx - np.asarray([s0, s1, s2])) // n
                    ok = np.all((q >= 0) & (q < ppa) & ((idx % n == 0) | (np.asarray([s0, s1, s2]) == 0)), axis=1)
                    live[tuple(q[ok].T)] = True
    return int(live.sum())


def oscillatory_2048_study(ctx, dev, steps=2):
    """The oscillatory charges of sec. 7.2 at 2048^3 (32^3-cell patches, L27,
    beta 3.25, four levels), the settings of Tables 12 (alpha 1.75 at every
    level) and 14 (1.75, 2, 2.25 from the finest level up), P = 1 and 4, float64
    local convolutions.  The plans keep per-patch buffers for the live patches
    only (max_live); the error is the scaled maximum over every node of the
    finest level against the closed form, evaluated on the device in slabs."""
    import torch
    from paper_1702_08111_amd import mlc as gm
    N, n = 2048, 32
    live = _osc_live_patches(N, n)
    cap = 1024
    progress(f"2048^3: {live} of {(N // n) ** 3} patches carry charge; buffers for {cap}")
    settings = [("table_14", (2.0, 2.25)), ("table_12", (1.75, 1.75))]
    probs = {(t, P): gm.problem(N, n, 1.75, 3.25, P, 6, conv="fp64", levels=4, level_alpha=la, max_live=cap)
             for t, la in settings for P in (1, 4)}
    ws_bytes = max(gm.problem_workspace_bytes(p) for p in probs.values())
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    f = torch.empty((N + 1,) * 3, dtype=torch.float64, device=dev)
    phi = torch.empty_like(f)
    ax = torch.arange(N + 1, dtype=torch.float64, device=dev) / N
    out = {"config": "oscillatory charges (sec. 7.2), 2048^3, 32^3-cell patches, L27, beta 3.25, 4 levels, float64 "
                     "local convolutions, charge sampled on the device from its radial terms, Boole moments "
                     "(error_gauss_moments: the moments integrated from the radial terms, 2 Gauss points per "
                     "cell); error = max over all nodes |phi - closed form| / max |closed form|",
           "live_patches": live, "max_live": cap, "workspace_GiB": ws_bytes / 2 ** 30}
    def scaled_error():
        err = scale = 0.0
        for k0 in range(0, N + 1, 8):
            k1 = min(k0 + 8, N + 1)
            exact = torch.zeros((k1 - k0, N + 1, N + 1), dtype=torch.float64, device=dev)
            for c in mi.OSC_CENTRES:
                r = torch.sqrt(((ax[k0:k1] - c[0]) ** 2)[:, None, None] + ((ax - c[1]) ** 2)[None, :, None]
                               + ((ax - c[2]) ** 2)[None, None, :]) / mi.OSC_RO
                exact += mi._osc_psi(r, xp=torch) / mi.OSC_RO
                del r
            err = max(err, float((phi[k0:k1] - exact).abs().max()))
            scale = max(scale, float(exact.abs().max()))
            del exact
        return err / scale

    for (table, P), prob in probs.items():
        plan = ctx.plan(prob)
        # the library samples the radial terms into f and integrates the
        # moments by Gauss quadrature (two points per cell); then plain solves
        # of that f (Boole moments of the node data)
        plan.solve_analytic(mi.oscillatory_terms(), 2, f, phi, ws)
        torch.cuda.synchronize()
        err_gauss = scaled_error()
        plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.solve(f, phi, ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        err = scaled_error()
        row = {"ms_per_step": ms, "value": N ** 3 / (ms * 1e-3), "unit": "grid points/s",
               "level_alpha": list(plan.info["level_alpha"][:2]), "error": err,
               "error_gauss_moments": err_gauss}
        out.setdefault(table, {})[f"P{P}"] = row
        progress(f"2048^3 {table} P={P}: {ms:.1f} ms/solve, error {err:.5e} (Gauss moments {err_gauss:.5e})")
        plan.close()
    del ws, f, phi
    torch.cuda.empty_cache()
    return out


SWEEP = [
    # (alpha, beta, P, Q, b): MLC-0 (beta = alpha) and MLC, the 19- and 27-point operators
    (1.5, 1.5, 4, 4, 2), (3.0, 3.0, 4, 4, 2), (1.5, 3.0, 4, 4, 2), (1.5, 6.0, 4, 4, 2), (3.0, 6.0, 4, 4, 2),
    (2.0, 2.0, 4, 6, 3), (1.5, 2.0, 4, 6, 2), (1.75, 3.25, 4, 6, 3), (1.75, 3.25, 9, 6, 3), (3.0, 6.0, 4, 6, 3),
]


def sweep_bench(ctx, dev, steps=3, N=256, n=32):
    """Cost and accuracy over (alpha, beta, P, Q) for the smooth charge of
    sec. 7.1 at 256^3 (32^3-cell patches): per setting the float64 and
    float32 solve times and errors against the closed form, and for one
    setting the same charge given analytically (Gauss-integrated moments)."""
    import torch
    from paper_1702_08111_amd import mlc as gm
    f = torch.from_numpy(mi.smooth_charge(N)).to(dev)
    exact = mi.smooth_potential(N)
    scale = np.abs(exact).max()
    rows = []
    for a, bt, P, Q, b in SWEEP:
        row = {"alpha": a, "beta": bt, "P": P, "Q": Q, "b": b, "mlc0": a == bt}
        for conv in ("fp64", "fp32"):
            plan = ctx.plan(gm.problem(N, n, a, bt, P, Q, b=b, conv=conv))
            ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
            phi = torch.empty_like(f)
            plan.solve(f, phi, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.solve(f, phi, ws)
            torch.cuda.synchronize()
            row[conv + "_ms"] = round((time.perf_counter() - t0) * 1e3 / steps, 3)
            row[conv + "_err"] = float(np.abs(phi.cpu().numpy() - exact).max() / scale)
            if conv == "fp64" and (a, bt, P, Q) == (1.75, 3.25, 4, 6):
                fa = torch.empty_like(f)
                plan.solve_analytic([(t[0], t[1], t[2], t[3], t[4]) for t in mi.smooth_terms()], 4, fa, phi, ws)
                torch.cuda.synchronize()
                row["fp64_gauss_moments_err"] = float(np.abs(phi.cpu().numpy() - exact).max() / scale)
            del ws
            plan.close()
        rows.append(row)
    torch.cuda.empty_cache()
    return {"config": f"smooth charge of sec. 7.1, {N}^3, {n}^3-cell patches; error = max|phi - closed form| / "
                      "max|closed form|", "rows": rows}


def serving_bench(ctx, count, load, dev, warm=50, sat_requests=120, pool=4, ring=32, verify_per_size=8):
    """The serving loop: requests with N ~ U{64,128,192,256}, n ~ U{16,32},
    Q ~ U{4,6}, 1-4 seeded bumps, float32 convolutions.  First the
    saturation rate (a burst of requests, drained); then Poisson arrivals at
    `load` x that rate, warm-ups then `count` measured requests.  Each (N)
    keeps `pool` charges (those of its first requests) reused cyclically and
    a ring of output arrays; plans are built up front (resident tables).
    Afterwards the results still in the rings (up to verify_per_size per N)
    are compared bit for bit with the same problems solved alone."""
    import torch
    from paper_1702_08111_amd import mlc as gm
    reqs = mi.serving_requests(warm + count + sat_requests, 1.0, seed=105)
    charges, outs = {}, {}
    for _, N, n, Q, b in reqs:
        lst = charges.setdefault(N, [])
        if len(lst) < pool:
            lst.append(torch.from_numpy(mi.bump_charge(N, b)).to(dev))
    for N in charges:
        outs[N] = [torch.empty((N + 1,) * 3, dtype=torch.float64, device=dev) for _ in range(ring)]
    torch.cuda.synchronize()
    srv = gm.Server(ctx, budget_bytes=48 << 30, streams=3, max_batch=8)
    probs = {}
    for _, N, n, Q, _ in reqs:
        if (N, n, Q) not in probs:
            probs[(N, n, Q)] = gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp32")
            srv.prepare(probs[(N, n, Q)])
    use = {N: 0 for N in charges}
    last = {}   # (N, ring slot) -> (n, Q, k) of the request that wrote it last

    def submit(N, n, Q):
        k = use[N]
        use[N] += 1
        st, t = srv.submit(probs[(N, n, Q)], charges[N][k % pool], outs[N][k % ring])
        assert st == gm.MLC_OK, st
        last[(N, k % ring)] = (n, Q, k)
        return t

    # saturation: a burst, drained
    burst = reqs[warm + count:]
    t0 = time.perf_counter()
    tickets = [submit(N, n, Q) for _, N, n, Q, _ in burst]
    srv.drain()
    sat_wall = time.perf_counter() - t0
    for t in tickets:
        srv.poll(t)
    sat_rate = len(burst) / sat_wall
    sat_points = sum(N ** 3 for _, N, _, _, _ in burst) / sat_wall
    # open loop at load x saturation: arrival times rescaled from the unit-rate stream
    rate = load * sat_rate
    stream = reqs[:warm + count]
    pending = {}
    done = []
    t0 = time.perf_counter()
    k = 0
    while k < len(stream) or pending:
        now = time.perf_counter() - t0
        while k < len(stream) and stream[k][0] / rate <= now:
            _, N, n, Q, _ = stream[k]
            pending[submit(N, n, Q)] = (k, N)
            k += 1
        for t in list(pending):
            r = srv.poll(t)
            if r is not None:
                kk, N = pending.pop(t)
                done.append((kk, N, r, time.perf_counter() - t0))
        if k < len(stream):
            wait = stream[k][0] / rate - (time.perf_counter() - t0)
            if wait > 2e-4:
                time.sleep(min(wait, 1e-3))
    srv.close()
    torch.cuda.synchronize()
    # the results still held in the output rings, each against the same
    # problem solved alone by its own plan (bit for bit)
    checked = equal = 0
    alone = {}
    for (N, slot), (n, Q, k) in sorted(last.items()):
        if slot >= verify_per_size:
            continue
        if (N, n, Q) not in alone:
            pl = ctx.plan(probs[(N, n, Q)])
            alone[(N, n, Q)] = (pl, torch.empty(pl.workspace_bytes, dtype=torch.uint8, device=dev))
        pl, ws = alone[(N, n, Q)]
        ref = torch.empty_like(outs[N][slot])
        pl.solve(charges[N][k % pool], ref, ws)
        torch.cuda.synchronize()
        checked += 1
        equal += int(torch.equal(ref, outs[N][slot]))
    for pl, _ in alone.values():
        pl.close()
    del alone
    meas = [d for d in done if d[0] >= warm]
    lat = np.array([d[2]["total_ms"] for d in meas])
    qms = np.array([d[2]["queue_ms"] for d in meas])
    bad = sum(1 for d in done if d[2]["status"] != 0)
    first = min(stream[d[0]][0] / rate for d in meas)
    last = max(d[3] for d in meas)
    points = sum(d[1] ** 3 for d in meas)
    del charges, outs
    torch.cuda.empty_cache()
    return {"value": points / (last - first), "unit": "grid points/s",
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "queue_p50_ms": float(np.percentile(qms, 50)), "queue_p99_ms": float(np.percentile(qms, 99)),
            "mean_batch": float(np.mean([d[2]["batch_size"] for d in meas])),
            "requests": len(meas), "warmup": warm, "failed": bad,
            "verified": checked, "verified_equal_alone": equal,
            "arrival_rate_rps": rate, "load": load, "saturation_rps": sat_rate,
            "saturation_points_per_s": sat_points,
            "config": "Poisson arrivals; N ~ U{64,128,192,256}, n ~ U{16,32}, Q ~ U{4,6}, 1-4 bumps (seed 105), "
                      "P=4, alpha=3, beta=6, fp32 convolutions; 3 streams, batches of <= 8, 48 GB arena"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the solver runs on a single "
              "GPU; sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1702_08111_amd import mlc as gm

    if args.paper_2048:
        study = oscillatory_2048_study(gm.Context(0), torch.device("cuda:0"))
        print(json.dumps({"study": "oscillatory_2048_four_levels", **study}), flush=True)
        return
    N, n, Q, bumps = mi.workload(args.workload)
    f_np = mi.bump_charge(N, bumps)
    exact = mi.bump_potential(N, bumps)
    dev = torch.device("cuda:0")
    f = torch.from_numpy(f_np).to(dev)
    ctx = gm.Context(0)
    p32 = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp32"))
    p64 = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv="fp64"))
    ws = torch.empty(max(p32.workspace_bytes, p64.workspace_bytes), dtype=torch.uint8, device=dev)
    phi32 = torch.empty_like(f)
    phi64 = torch.empty_like(f)
    stream = torch.cuda.current_stream()

    def timed(plan, phi, steps, warmup, timing):
        for _ in range(warmup):
            plan.solve(f, phi, ws, stream)
        torch.cuda.synchronize()
        if timing:
            plan.set_timing(True)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            plan.solve(f, phi, ws, stream)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        kt = plan.timing() if timing else {}
        if timing:
            plan.set_timing(False)
        return (t1 - t0) * 1e3 / steps, lat, kt

    progress(f"plans built; timing {args.steps} float32-convolution solves")
    ms32, lat32, kt32 = timed(p32, phi32, args.steps, args.warmup, True)
    progress(f"float32 {ms32:.3f} ms/solve; timing {args.fp64_steps} float64 solves")
    ms64, lat64, _ = timed(p64, phi64, args.fp64_steps, 1, False)
    progress(f"float64 {ms64:.3f} ms/solve")
    # the same workload with empty patches skipped (exact: an empty patch's
    # local field and moments are zero); reported beside the dense figure
    sparse = {}
    for conv, ref, steps in () if args.no_sparse else (("fp32", phi32, args.steps), ("fp64", phi64, args.fp64_steps)):
        ps = ctx.plan(gm.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, skip_empty=1))
        wss = torch.empty(ps.workspace_bytes, dtype=torch.uint8, device=dev)
        phis = torch.empty_like(f)
        for _ in range(max(1, args.warmup)):
            ps.solve(f, phis, wss, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ps.solve(f, phis, wss, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        sparse[conv] = {"ms_per_step": ms, "value": N ** 3 / (ms * 1e-3), "unit": "grid points/s",
                        "equal_to_dense": bool(torch.equal(phis, ref))}
        del wss, phis
        ps.close()
    if sparse:
        sparse["note"] = ("mlc_problem.skip_empty = 1: patches whose node charge is all zero skip their local "
                          "convolutions (found on the device every solve); phi equal to the dense solve element for "
                          "element")
        progress(f"empty patches skipped: float32 {sparse['fp32']['ms_per_step']:.3f} ms, "
                 f"float64 {sparse['fp64']['ms_per_step']:.3f} ms")
    else:
        sparse = None
    a32, a64 = phi32.cpu().numpy(), phi64.cpu().numpy()
    scale = np.abs(a64).max()
    err_32_64 = float(np.abs(a32 - a64).max() / scale)
    err64_exact = float(np.abs(a64 - exact).max() / np.abs(exact).max())
    err32_exact = float(np.abs(a32 - exact).max() / np.abs(exact).max())
    errors = {"fp32_vs_fp64_relmax": err_32_64, "fp64_vs_closed_form": err64_exact,
              "fp32_vs_closed_form": err32_exact, "fp32_vs_oracle": None, "fp64_vs_oracle": None}

    # roofline of the dominant kernel (largest measured time per solve)
    model = kernel_model(p32.info)
    # ms per solve of each kernel (a kernel may be launched once per patch chunk)
    per_kernel = {k: v[1] / args.steps for k, v in kt32.items()}
    launches = {k: v[0] / args.steps for k, v in kt32.items()}
    # (the longest kernel the model covers; at 256^3 it is the longest of all)
    longest = max(per_kernel, key=per_kernel.get)
    modeled = [k for k in per_kernel if k in model]
    dom = max(modeled, key=per_kernel.get) if modeled else longest
    roof = None
    if dom in model:
        t = per_kernel[dom] * 1e-3
        gbs = model[dom]["bytes"] / t / 1e9
        tfs = model[dom]["flops"] / t / 1e12
        if gbs / HBM_PEAK_GBS >= tfs / FP32_PEAK_TFLOPS:
            roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None}
        else:
            roof = {"bound": "alu", "achieved": round(tfs, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tfs / FP32_PEAK_TFLOPS, 4), "traffic": None}
        roof["kernel"] = dom
        roof["longest_kernel"] = longest
        roof["launches_per_solve"] = launches[dom]
        roof["ms_per_launch"] = round(per_kernel[dom] / launches[dom], 4)
        tr = measured_traffic(dom, args.workload)
        roof["traffic"] = tr
        roof["algorithmic_bytes_per_launch"] = model[dom]["bytes"] / launches[dom]

    # whole-solve fractions of the HBM and fp32 vector roofs (model above)
    sb, sf = solve_model(p32.info)
    t32 = ms32 * 1e-3
    solve_roof = {"bytes_model": sb, "flops_model": sf,
                  "hbm_frac": round(sb / t32 / (HBM_PEAK_GBS * 1e9), 4),
                  "alu_frac": round(sf / t32 / (FP32_PEAK_TFLOPS * 1e12), 4),
                  "basis": "compulsory bytes with one round trip of the pruned spectral intermediates; "
                           "nominal FFT flops; fp32 vector peak"}

    if args.copy_calibration:
        src = torch.empty(256 * 1024 * 1024, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    if args.batch_steps > 0:
        progress("uneven 64-problem batch")
    batch = batch_bench(ctx, args.batch_steps, dev) if args.batch_steps > 0 else None
    sweep = None
    if not args.no_sweep:
        progress("(alpha, beta, P, Q) sweep, 256^3 smooth charge")
        sweep = sweep_bench(ctx, dev)
    osc = None
    if args.osc_steps > 0:
        progress("oscillatory workload, 384^3")
        osc = oscillatory_bench(ctx, args.osc_steps, dev)
    ml = None
    if args.ml_steps > 0:
        progress("multilevel: smooth charge, 512^3, three levels")
        ml = multilevel_bench(ctx, args.ml_steps, dev)
    if args.serve_requests > 0:
        progress("serving loop")
    serving = serving_bench(ctx, args.serve_requests, args.serve_load, dev) if args.serve_requests > 0 else None

    cpu = cpu_direct = None
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline")
        cpu, phi_or = cpu_baseline(args.workload)
        oscale = np.abs(phi_or).max()
        errors["fp32_vs_oracle"] = float(np.abs(a32 - phi_or).max() / oscale)
        errors["fp64_vs_oracle"] = float(np.abs(a64 - phi_or).max() / oscale)
        errors["fp32_within_2e-6_of_oracle"] = errors["fp32_vs_oracle"] < 2e-6
        errors["fp64_within_1e-12_of_oracle"] = errors["fp64_vs_oracle"] < 1e-12
        del phi_or
        progress("CPU oracle baseline, literal-sum convolutions")
        cpu_direct = cpu_baseline_direct()

    value = N ** 3 / (ms32 * 1e-3)
    line = {
        "metric": "grid points/s per MLC solve at 256^3, FP32 vs FP64 at stated err; p50/p99 latency",
        "value": value,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_detail": "f32 local convolutions (the dominant kernels); f64 moments, far fields, coarse solve, "
                        "boundary values, Dirichlet solves",
        "data": "synthetic",
        "config": {"workload": f"two-level MLC, {N}^3 cells, {n}^3-cell patches ({N // n}^3 = "
                               f"{(N // n) ** 3}), L{19 if Q == 4 else 27} (Q={Q}), alpha=3, beta=6, P=4, "
                               f"{len(bumps)} seeded compact bumps",
                   "N": N, "patch": n, "Q": Q, "alpha": 3.0, "beta": 6.0, "P": 4,
                   "fft_size": p32.info["M"], "coarse_fft": p32.info["M_coarse"]},
        "p50_ms": float(np.percentile(lat32, 50)),
        "p99_ms": float(np.percentile(lat32, 99)),
        "fp64": {"value": N ** 3 / (ms64 * 1e-3), "ms_per_step": ms64,
                 "p50_ms": float(np.percentile(lat64, 50)), "p99_ms": float(np.percentile(lat64, 99))},
        "error": errors,
        "kernels_ms": {k: round(v, 4) for k, v in sorted(per_kernel.items(), key=lambda kv: -kv[1])},
        "roofline": roof,
        "solve_roofline": solve_roof,
        "cpu_baseline": cpu,
        "cpu_baseline_direct": cpu_direct,
        "sparse": sparse,
        "batch": batch,
        "oscillatory": osc,
        "multilevel": ml,
        "sweep": sweep,
        "serving": serving,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
