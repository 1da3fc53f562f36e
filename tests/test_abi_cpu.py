"""Host-side checks of the C ABI (no device work): the library loads,
exports every function include/mlc.h declares, and validates problems."""
import os
import re

import pytest

from paper_1702_08111_amd import mlc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "mlc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlc_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = mlc.lib()
    names = _header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(mlc._SIGS), "binding and header disagree"


def test_status_strings():
    assert mlc.status_string(0) == "MLC_OK"
    assert mlc.status_string(-2) == "MLC_ERR_UNSUPPORTED"


@pytest.mark.parametrize("name,N,n,Q,fft,expect", [
    ("32^3 plain", 32, 8, 4, 0, dict(d_alpha=8, d_beta=20, e=16, M=50, Wc=11, Wa=25, nplanes_a=4, Ns=19, No=13)),
    ("128^3", 128, 16, 4, 96, dict(d_alpha=16, d_beta=40, e=24, M=96, Wc=17, Wa=49, Ns=53, No=37, M_coarse=90)),
    ("256^3 L27", 256, 32, 6, 0, dict(d_alpha=32, d_beta=80, e=44, M=160, Wc=31, Wa=97, nplanes_a=4, Ns=105,
                                        No=71, M_coarse=180, npatch=512, M_table=250)),
])
def test_derived_sizes(name, N, n, Q, fft, expect):
    info = mlc.problem_info(mlc.problem(N, n, 3.0, 6.0, 4, Q, conv="fp32", fft_size=fft))
    for k, v in expect.items():
        assert info[k] == v, (k, info[k], v)
    assert info["K"] == 20


@pytest.mark.parametrize("kw,status", [
    (dict(N=30, n=8), mlc.MLC_ERR_INVALID_ARG),          # N % n
    (dict(N=36, n=6), mlc.MLC_ERR_INVALID_ARG),          # n % 4
    (dict(N=32, n=8, alpha=3, beta=2), mlc.MLC_ERR_INVALID_ARG),
    (dict(N=32, n=8, Q=5), mlc.MLC_ERR_UNSUPPORTED),
    (dict(N=32, n=8, P=10), mlc.MLC_ERR_UNSUPPORTED),
    (dict(N=32, n=8, alpha=1.5, beta=1.5), mlc.MLC_ERR_UNSUPPORTED),   # margin 2 not a multiple of 4
    (dict(N=32, n=8, fft_size=40), mlc.MLC_ERR_INVALID_ARG),           # below 2(n+e)+1
    (dict(N=32, n=8, Z=100), mlc.MLC_ERR_UNSUPPORTED),
    (dict(N=32, n=8, rhs_order=5), mlc.MLC_ERR_INVALID_ARG),
    (dict(N=32, n=8, skip_empty=2), mlc.MLC_ERR_INVALID_ARG),
    (dict(N=(64, 40, 32), n=16), mlc.MLC_ERR_INVALID_ARG),      # a box edge not a multiple of n
    (dict(N=(64, 0, 32), n=16), mlc.MLC_ERR_INVALID_ARG),
    (dict(N=32, n=8, Q=4, rhs_order=6), mlc.MLC_ERR_UNSUPPORTED),      # the 27-point operator's
    (dict(N=64, n=8, levels=3, level_alpha=(3.5,)), mlc.MLC_ERR_UNSUPPORTED),  # level-1 margin 10
    (dict(N=64, n=8, levels=3, level_alpha=(0.5,)), mlc.MLC_ERR_INVALID_ARG),    # below 1
    (dict(N=64, n=8, alpha=2.0, beta=3.0, levels=3, level_alpha=(4.0,)), mlc.MLC_ERR_INVALID_ARG),  # above beta
])
def test_validation(kw, status):
    args = dict(N=32, n=8, alpha=3.0, beta=6.0, P=4, Q=4)
    args.update(kw)
    with pytest.raises(mlc.MLCError) as ei:
        mlc.problem_info(mlc.problem(**args))
    assert ei.value.status == status


def test_context_without_device_fails_cleanly():
    """Without a usable GPU the context call reports MLC_ERR_DEVICE instead
    of crashing; with one it succeeds."""
    import ctypes
    h = ctypes.c_void_p()
    st = mlc.lib().mlc_context_create(0, 0, ctypes.byref(h))
    assert st in (mlc.MLC_OK, mlc.MLC_ERR_DEVICE)
    if st == mlc.MLC_OK:
        mlc.lib().mlc_context_destroy(h)


def test_problem_workspace_bytes_host_only():
    """Workspace sizing needs no device; it covers at least phi^B on all
    nodes and the Dirichlet work arrays of every patch, and grows with N."""
    sizes = []
    for N in (64, 128, 256):
        prob = mlc.problem(N, 32, 3.0, 6.0, 4, 6, conv="fp32")
        b = mlc.problem_workspace_bytes(prob)
        npatch = (N // 32) ** 3
        assert b >= (N + 1) ** 3 * 8 + npatch * 31 ** 3 * 8
        assert b % 256 == 0
        sizes.append(b)
    assert sizes[0] < sizes[1] < sizes[2]
    with pytest.raises(mlc.MLCError):
        mlc.problem_workspace_bytes(mlc.problem(100, 32, 3.0, 6.0, 4, 6))


def test_server_calls_reject_null_handles():
    """Every serving call validates its handle before touching a device."""
    import ctypes
    L = mlc.lib()
    h = ctypes.c_void_p()
    assert L.mlc_server_create(None, None, ctypes.byref(h)) == mlc.MLC_ERR_INVALID_ARG
    prob = mlc.problem(32, 8)
    t = ctypes.c_uint64()
    assert L.mlc_server_submit(None, ctypes.byref(prob), 1, 1, ctypes.byref(t)) == mlc.MLC_ERR_INVALID_ARG
    done = ctypes.c_int32()
    assert L.mlc_server_poll(None, 1, ctypes.byref(done), None) == mlc.MLC_ERR_INVALID_ARG
    assert L.mlc_server_prepare(None, ctypes.byref(prob)) == mlc.MLC_ERR_INVALID_ARG
    assert L.mlc_server_drain(None) == mlc.MLC_ERR_INVALID_ARG
    assert L.mlc_server_destroy(None) == mlc.MLC_ERR_INVALID_ARG


def test_fft_size_autotune_flag():
    """fft_size = -1 (autotune) validates like 0; below -1 is rejected."""
    a = mlc.problem_info(mlc.problem(64, 16, 3.0, 6.0, 4, 4, fft_size=-1))
    b = mlc.problem_info(mlc.problem(64, 16, 3.0, 6.0, 4, 4, fft_size=0))
    assert a["M"] == b["M"] == 90
    with pytest.raises(mlc.MLCError) as ei:
        mlc.problem_info(mlc.problem(64, 16, 3.0, 6.0, 4, 4, fft_size=-2))
    assert ei.value.status == mlc.MLC_ERR_INVALID_ARG


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    """No CPU fallback: without the built library every call raises."""
    monkeypatch.setattr(mlc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(mlc, "_lib", None)
    with pytest.raises(RuntimeError):
        mlc.problem_info(mlc.problem(32, 8))
    with pytest.raises(RuntimeError):
        mlc.Context(0)


@pytest.mark.parametrize("N,n,Q,conv", [(64, 16, 4, "fp32"), (128, 32, 6, "fp32"), (64, 16, 6, "fp64")])
def test_autotuned_workspace_bounds_every_candidate(N, n, Q, conv):
    """With fft_size = -1 the host-side workspace figure is the largest over
    every built torus the autotuner may pick, so a server sizing requests by
    it never under-reserves for the tuned plan."""
    tuned = mlc.problem_workspace_bytes(mlc.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, fft_size=-1))
    sizes = []
    for M in (50, 64, 72, 90, 96, 120, 128, 150, 160, 180, 192):
        try:
            sizes.append(mlc.problem_workspace_bytes(mlc.problem(N, n, 3.0, 6.0, 4, Q, conv=conv, fft_size=M)))
        except mlc.MLCError:
            pass
    assert len(sizes) >= 2
    assert tuned == max(sizes)


def test_sixth_order_sizes():
    """rhs_order 6 adds the modified right-hand side, (N+1)^3 doubles, to the
    workspace and nothing else; the info reports the order."""
    base = mlc.problem(32, 8, 3.0, 6.0, 4, 6, conv="fp64", Z=64)
    six = mlc.problem(32, 8, 3.0, 6.0, 4, 6, conv="fp64", Z=64, rhs_order=6)
    assert mlc.problem_info(base)["rhs_order"] == 4 and mlc.problem_info(six)["rhs_order"] == 6
    extra = mlc.problem_workspace_bytes(six) - mlc.problem_workspace_bytes(base)
    assert 33 ** 3 * 8 <= extra < 33 ** 3 * 8 + 512


def test_box_domain_sizes():
    """A box is solved in the smallest cube the plan can run: N a multiple of
    n (two levels) or of 4n (three levels); the info reports both, and the
    origin as given; n_cells and box_cells together are refused."""
    i = mlc.problem_info(mlc.problem((64, 48, 32), 16, 3.0, 6.0, 4, 4, origin=(1.0, -2.0, 0.5)))
    assert i["N"] == 64 and i["box"] == [64, 48, 32] and i["origin"] == [1.0, -2.0, 0.5]
    assert mlc.problem_info(mlc.problem((80, 16, 16), 16, levels=3))["N"] == 128
    assert mlc.problem_info(mlc.problem(64, 16))["box"] == [64, 64, 64]
    p = mlc.problem((64, 48, 32), 16)
    p.n_cells = 64
    with pytest.raises(mlc.MLCError) as ei:
        mlc.problem_info(p)
    assert ei.value.status == mlc.MLC_ERR_INVALID_ARG
    # the workspace holds f and phi in the enclosing cube besides the cube's own
    extra = mlc.problem_workspace_bytes(mlc.problem((64, 48, 32), 16)) - mlc.problem_workspace_bytes(mlc.problem(64, 16))
    assert 2 * 65 ** 3 * 8 <= extra < 2 * 65 ** 3 * 8 + 1024


def test_max_live_sizes():
    """max_live keeps per-patch convolution buffers for that many patches only
    (at most npatch) and turns on skip_empty; the Dirichlet work array is
    chunked at 4 GB, so at 2048^3 with four levels the workspace fits one GPU
    beside f and phi."""
    base = mlc.problem(128, 16, 3.0, 6.0, 4, 4)
    cap = mlc.problem(128, 16, 3.0, 6.0, 4, 4, max_live=40)
    ib, ic = mlc.problem_info(base), mlc.problem_info(cap)
    assert ib["slots"] == ib["npatch"] == 512 and ib["skip_empty"] == 0
    assert ic["slots"] == 40 and ic["skip_empty"] == 1
    assert mlc.problem_workspace_bytes(cap) < mlc.problem_workspace_bytes(base) / 2
    assert mlc.problem_info(mlc.problem(128, 16, max_live=10 ** 6))["slots"] == 512
    with pytest.raises(mlc.MLCError) as ei:
        mlc.problem_info(mlc.problem(128, 16, max_live=-1))
    assert ei.value.status == mlc.MLC_ERR_INVALID_ARG
    big = mlc.problem(2048, 32, 1.75, 3.25, 4, 6, conv="fp32", levels=4, level_alpha=(2.0, 2.25), max_live=4096)
    ws = mlc.problem_workspace_bytes(big)
    nodes = 8 * 2049 ** 3
    assert ws + 2 * nodes < 270 * 2 ** 30, ws / 2 ** 30


def test_grid_launch_limit():
    """The skeleton kernels take one thread per skeleton node in one launch:
    grids whose skeleton reaches 2^31 nodes are refused as unsupported."""
    assert mlc.problem_info(mlc.problem(2048, 32, 1.75, 3.25, 4, 6, levels=4, max_live=1024))["N"] == 2048
    with pytest.raises(mlc.MLCError) as ei:
        mlc.problem_info(mlc.problem(4096, 32, 1.75, 3.25, 4, 6, levels=4, max_live=1024))
    assert ei.value.status == mlc.MLC_ERR_UNSUPPORTED
