"""ctypes binding of libmlc (include/mlc.h).  Argument marshalling only:
every step of a solve runs in the library's HIP kernels.

Device arrays are passed as torch CUDA tensors (their data_ptr()) or as raw
integers; streams as torch.cuda.Stream or raw hipStream_t integers.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# MLC_LIBRARY names another build of the same library (e.g. the
# host-sanitized libmlc_san.so for the CPU-side ABI checks)
LIB_PATH = os.environ.get("MLC_LIBRARY") or os.path.join(_HERE, "libmlc.so")

MLC_OK = 0
MLC_ERR_INVALID_ARG = -1
MLC_ERR_UNSUPPORTED = -2
MLC_ERR_OUT_OF_MEMORY = -3
MLC_ERR_DEVICE = -4
MLC_ERR_BUSY = -5
MLC_ERR_NOT_READY = -6

MLC_CONV_FP64 = 0
MLC_CONV_FP32 = 1

MLC_STATIC_SCRATCH_BYTES = 512 << 20   # include/mlc.h

MLC_VIEW_MOMENTS = 0
MLC_VIEW_COARSE_RHS = 1
MLC_VIEW_COARSE_PHI = 2
MLC_VIEW_BOUNDARY = 3
MLC_VIEW_LOCAL_COARSE = 4
MLC_VIEW_LOCAL_PLANES = 5
MLC_VIEW_LEVEL_CHARGE = 6
MLC_VIEW_LEVEL_PHI = 7
MLC_VIEW_LEVEL_WORKSPACE = 8
MLC_VIEW_CHARGE = 9


class mlc_problem(ctypes.Structure):
    _fields_ = [
        ("n_cells", ctypes.c_int32),
        ("h", ctypes.c_double),
        ("patch", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("P", ctypes.c_int32),
        ("Q", ctypes.c_int32),
        ("interp_b", ctypes.c_int32),
        ("conv_precision", ctypes.c_int32),
        ("fft_size", ctypes.c_int32),
        ("dgf_half_width", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("level_alpha", ctypes.c_double * 3),
        ("rhs_order", ctypes.c_int32),
        ("skip_empty", ctypes.c_int32),
        ("box_cells", ctypes.c_int32 * 3),
        ("origin", ctypes.c_double * 3),
        ("max_live", ctypes.c_int32),
    ]


MLC_PROFILE_BUMP = 0
MLC_PROFILE_SMOOTH = 1
MLC_PROFILE_OSCILLATORY = 2
MLC_MAX_RADIAL_TERMS = 16


class mlc_radial_charge(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_double * 3), ("radius", ctypes.c_double), ("weight", ctypes.c_double),
                ("param", ctypes.c_double), ("profile", ctypes.c_int32)]


class mlc_plan_info(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "N", "n", "P", "Q", "b", "K", "d_alpha", "d_beta", "e", "patches_per_axis", "npatch",
        "M", "M_coarse", "M_table", "Wc", "Wa", "nplanes_a", "S_lo", "Ns", "O_lo", "No", "Z",
        "conv_precision")] + [("h", ctypes.c_double), ("H", ctypes.c_double), ("out_planes", ctypes.c_int32),
                              ("levels", ctypes.c_int32), ("level_margin", ctypes.c_int32),
                              ("level_N", ctypes.c_int32), ("alpha", ctypes.c_double),
                              ("beta", ctypes.c_double), ("level_alpha", ctypes.c_double * 3),
                              ("rhs_order", ctypes.c_int32), ("skip_empty", ctypes.c_int32),
                              ("box", ctypes.c_int32 * 3), ("origin", ctypes.c_double * 3),
                              ("slots", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("level_alpha", "box", "origin"):
            d[k] = list(d[k])
        return d


class mlc_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


class mlc_server_config(ctypes.Structure):
    _fields_ = [("workspace_budget_bytes", ctypes.c_size_t), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_queue", ctypes.c_int32)]


class mlc_timing(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("device_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol declared in include/mlc.h, with its ctypes signature
_P = ctypes.c_void_p
_SIGS = {
    "mlc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mlc_problem_info": (ctypes.c_int, [ctypes.POINTER(mlc_problem), ctypes.POINTER(mlc_plan_info)]),
    "mlc_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "mlc_context_destroy": (ctypes.c_int, [_P]),
    "mlc_last_error": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "mlc_plan_create": (ctypes.c_int, [_P, ctypes.POINTER(mlc_problem), ctypes.POINTER(_P)]),
    "mlc_plan_destroy": (ctypes.c_int, [_P]),
    "mlc_plan_get_info": (ctypes.c_int, [_P, ctypes.POINTER(mlc_plan_info)]),
    "mlc_plan_workspace_bytes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "mlc_problem_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(mlc_problem), ctypes.POINTER(ctypes.c_size_t)]),
    "mlc_solve": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_size_t, _P]),
    "mlc_solve_static": (ctypes.c_int, [_P, _P, _P, _P]),
    "mlc_solve_analytic": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(mlc_radial_charge), ctypes.c_int32,
                                          _P, _P, _P, ctypes.c_size_t, _P]),
    "mlc_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_size_t)]),
    "mlc_solve_batched": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                         _P, ctypes.c_size_t, _P]),
    "mlc_graph_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P),
                                        _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "mlc_graph_launch": (ctypes.c_int, [_P, _P]),
    "mlc_graph_destroy": (ctypes.c_int, [_P]),
    "mlc_plan_coarse_level": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "mlc_workspace_view": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_size_t)]),
    "mlc_dgf_table": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_P)]),
    "mlc_plan_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "mlc_plan_timing": (ctypes.c_int, [_P, ctypes.POINTER(mlc_kernel_time), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "mlc_server_create": (ctypes.c_int, [_P, ctypes.POINTER(mlc_server_config), ctypes.POINTER(_P)]),
    "mlc_server_prepare": (ctypes.c_int, [_P, ctypes.POINTER(mlc_problem)]),
    "mlc_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(mlc_problem), _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "mlc_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(mlc_timing)]),
    "mlc_server_drain": (ctypes.c_int, [_P]),
    "mlc_server_destroy": (ctypes.c_int, [_P]),
}

_lib = None


def lib():
    """The loaded libmlc; raises if the library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MLCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


def status_string(s):
    return lib().mlc_status_string(s).decode()


def _check(status, ctx=None):
    if status != MLC_OK:
        buf = ctypes.create_string_buffer(512)
        lib().mlc_last_error(ctx, buf, 512)
        raise MLCError(status, buf.value.decode())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def problem(N, n, alpha=3.0, beta=6.0, P=4, Q=4, b=0, h=None, conv="fp32", fft_size=0, Z=0, levels=0,
            level_alpha=(), rhs_order=0, skip_empty=0, origin=(0.0, 0.0, 0.0), max_live=0):
    """N: cells per axis of a cube, or a triple (B0, B1, B2) for a box domain
    (h then defaults to 1 / max B_d)."""
    la = list(level_alpha) + [0.0] * (3 - len(level_alpha))
    if isinstance(N, (tuple, list)):
        box, ncells = [int(x) for x in N], 0
        hh = (1.0 / max(box)) if h is None else h
    else:
        box, ncells = [0, 0, 0], int(N)
        hh = (1.0 / N) if h is None else h
    return mlc_problem(ncells, hh, n, alpha, beta, P, Q, b,
                       MLC_CONV_FP32 if conv == "fp32" else MLC_CONV_FP64, fft_size, Z, levels,
                       (ctypes.c_double * 3)(*la[:3]), rhs_order, skip_empty, (ctypes.c_int32 * 3)(*box),
                       (ctypes.c_double * 3)(*[float(x) for x in origin]), max_live)


def problem_workspace_bytes(prob):
    n = ctypes.c_size_t()
    _check(lib().mlc_problem_workspace_bytes(ctypes.byref(prob), ctypes.byref(n)))
    return n.value


def problem_info(prob):
    info = mlc_plan_info()
    _check(lib().mlc_problem_info(ctypes.byref(prob), ctypes.byref(info)))
    return info.as_dict()


class Context:
    def __init__(self, device=0, hbm_budget=0):
        h = ctypes.c_void_p()
        _check(lib().mlc_context_create(device, hbm_budget, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().mlc_context_destroy(self.handle)
            self.handle = None

    def dgf_table(self, Q, Z=128):
        p = ctypes.c_void_p()
        _check(lib().mlc_dgf_table(self.handle, Q, Z, ctypes.byref(p)), self.handle)
        return p.value

    def plan(self, prob):
        return Plan(self, prob)


class Plan:
    def __init__(self, ctx, prob):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib().mlc_plan_create(ctx.handle, ctypes.byref(prob), ctypes.byref(h)), ctx.handle)
        self.handle = h
        info = mlc_plan_info()
        _check(lib().mlc_plan_get_info(h, ctypes.byref(info)), ctx.handle)
        self.info = info.as_dict()
        nb = ctypes.c_size_t()
        _check(lib().mlc_plan_workspace_bytes(h, ctypes.byref(nb)), ctx.handle)
        self.workspace_bytes = nb.value

    def close(self):
        if self.handle:
            lib().mlc_plan_destroy(self.handle)
            self.handle = None

    def solve(self, f, phi, workspace, stream=None):
        """Enqueue one solve; f, phi, workspace are device tensors/pointers."""
        nbytes = workspace.numel() * workspace.element_size() if hasattr(workspace, "numel") else self.workspace_bytes
        _check(lib().mlc_solve(self.handle, _ptr(f), _ptr(phi), _ptr(workspace), nbytes, _stream(stream)),
               self.ctx.handle)

    def solve_static(self, f, phi, stream=None):
        """Enqueue one solve on the library's static scratch (no workspace,
        no device allocation); raises MLCError(MLC_ERR_UNSUPPORTED) when the
        plan's workspace exceeds it."""
        _check(lib().mlc_solve_static(self.handle, _ptr(f), _ptr(phi), _stream(stream)), self.ctx.handle)

    def solve_analytic(self, terms, gauss_points, f, phi, workspace, stream=None):
        """Enqueue one solve of a charge given as radial terms [(centre, radius,
        weight, param, profile)]: the library samples it into f (device
        array, overwritten) and takes the moments by Gauss integration."""
        arr = (mlc_radial_charge * len(terms))()
        for k, (c, R, w, prm, prof) in enumerate(terms):
            arr[k].centre[:] = [float(v) for v in c]
            arr[k].radius, arr[k].weight, arr[k].param, arr[k].profile = float(R), float(w), float(prm), int(prof)
        nbytes = workspace.numel() * workspace.element_size()
        _check(lib().mlc_solve_analytic(self.handle, len(terms), arr, gauss_points, _ptr(f), _ptr(phi),
                                        _ptr(workspace), nbytes, _stream(stream)), self.ctx.handle)

    def set_timing(self, enable):
        _check(lib().mlc_plan_set_timing(self.handle, 1 if enable else 0), self.ctx.handle)

    def timing(self):
        """{kernel name: (launches, total ms)} since timing was enabled."""
        arr = (mlc_kernel_time * 64)()
        cnt = ctypes.c_int32()
        _check(lib().mlc_plan_timing(self.handle, arr, 64, ctypes.byref(cnt)), self.ctx.handle)
        return {arr[k].name.decode(): (arr[k].launches, arr[k].total_ms) for k in range(min(cnt.value, 64))}

    def coarse_level(self):
        """The plan of the next coarser level of a multilevel plan (a
        read-only view: owned by this plan)."""
        h = ctypes.c_void_p()
        _check(lib().mlc_plan_coarse_level(self.handle, ctypes.byref(h)), self.ctx.handle)
        return _PlanView(self.ctx, h)

    def view(self, workspace, which):
        """(device pointer, bytes) of an intermediate held in the workspace."""
        p = ctypes.c_void_p()
        n = ctypes.c_size_t()
        _check(lib().mlc_workspace_view(self.handle, _ptr(workspace), which, ctypes.byref(p), ctypes.byref(n)),
               self.ctx.handle)
        return p.value, n.value


class _PlanView(Plan):
    """A plan owned by another plan (a coarser level): info and views only."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle
        info = mlc_plan_info()
        _check(lib().mlc_plan_get_info(handle, ctypes.byref(info)), ctx.handle)
        self.info = info.as_dict()
        nb = ctypes.c_size_t()
        _check(lib().mlc_plan_workspace_bytes(handle, ctypes.byref(nb)), ctx.handle)
        self.workspace_bytes = nb.value

    def close(self):
        self.handle = None


def solve_batched(plans, fs, phis, workspace, stream=None):
    k = len(plans)
    PA = ctypes.c_void_p * k
    hp = PA(*[p.handle.value for p in plans])
    fp = PA(*[_ptr(x) for x in fs])
    pp = PA(*[_ptr(x) for x in phis])
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib().mlc_solve_batched(k, hp, fp, pp, _ptr(workspace), nbytes, _stream(stream)), plans[0].ctx.handle)


class BatchGraph:
    """One batched solve captured into a HIP graph (mlc_graph_*): launch()
    replays it; the plans, arrays and workspace stay bound to it."""

    def __init__(self, plans, fs, phis, workspace):
        k = len(plans)
        PA = ctypes.c_void_p * k
        hp = PA(*[p.handle.value for p in plans])
        fp = PA(*[_ptr(x) for x in fs])
        pp = PA(*[_ptr(x) for x in phis])
        nbytes = workspace.numel() * workspace.element_size()
        h = ctypes.c_void_p()
        self.ctx = plans[0].ctx
        _check(lib().mlc_graph_create(k, hp, fp, pp, _ptr(workspace), nbytes, ctypes.byref(h)), self.ctx.handle)
        self.handle = h
        self._keep = (plans, fs, phis, workspace)

    def launch(self, stream=None):
        _check(lib().mlc_graph_launch(self.handle, _stream(stream)), self.ctx.handle)

    def close(self):
        if self.handle:
            lib().mlc_graph_destroy(self.handle)
            self.handle = None
            self._keep = None


def batch_workspace_bytes(plans):
    k = len(plans)
    PA = ctypes.c_void_p * k
    hp = PA(*[p.handle.value for p in plans])
    n = ctypes.c_size_t()
    _check(lib().mlc_batch_workspace_bytes(k, hp, ctypes.byref(n)))
    return n.value


class Server:
    """Request loop over a context (mlc_server_*): submit() queues a solve and
    returns a ticket; poll() reports it; the server's thread batches and
    launches requests on its own streams."""

    def __init__(self, ctx, budget_bytes=0, streams=0, max_batch=0, max_queue=0):
        self.ctx = ctx
        cfg = mlc_server_config(budget_bytes, streams, max_batch, max_queue)
        h = ctypes.c_void_p()
        _check(lib().mlc_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), ctx.handle)
        self.handle = h

    def prepare(self, prob):
        _check(lib().mlc_server_prepare(self.handle, ctypes.byref(prob)), self.ctx.handle)

    def submit(self, prob, f, phi):
        """Returns (status, ticket); status MLC_ERR_BUSY when the queue is full."""
        t = ctypes.c_uint64()
        st = lib().mlc_server_submit(self.handle, ctypes.byref(prob), _ptr(f), _ptr(phi), ctypes.byref(t))
        if st not in (MLC_OK, MLC_ERR_BUSY):
            _check(st, self.ctx.handle)
        return st, t.value

    def poll(self, ticket):
        """None while pending, else the timing dict (with the solve's status)."""
        done = ctypes.c_int32()
        tm = mlc_timing()
        st = lib().mlc_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(tm))
        if st == MLC_ERR_NOT_READY:
            return None
        if not done.value:
            _check(st, self.ctx.handle)
        return tm.as_dict()

    def drain(self):
        _check(lib().mlc_server_drain(self.handle), self.ctx.handle)

    def close(self):
        if self.handle:
            lib().mlc_server_destroy(self.handle)
            self.handle = None
