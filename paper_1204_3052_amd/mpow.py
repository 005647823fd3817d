"""Python binding of libmpow (ctypes).

Argument marshalling only: every function below forwards to the C entry point
of the same name declared in include/mpow.h, and every step of the power runs
in the library's HIP kernels.  PyTorch is used only to hand over device memory
(``tensor.data_ptr()``) and streams (``torch.cuda.current_stream()``).  If the
library has not been built, the first call raises - there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpow.so")

MPOW_SUCCESS = 0
MPOW_ERR_INVALID = 1
MPOW_ERR_UNSUPPORTED = 2
MPOW_ERR_NOMEM = 3
MPOW_ERR_DEVICE = 4
MPOW_ERR_BUDGET = 5
MPOW_ERR_TIMEOUT = 6

MPOW_FP32 = 0
MPOW_FP16X3 = 1
MPOW_BF16X3 = 2
MPOW_BF16X6 = 3

MPOW_FLAG_TIMING = 1
MPOW_FLAG_POISON = 2
MPOW_FLAG_EXPM = 4
MPOW_FLAG_WINDOW = 8
MPOW_FLAG_SPLIT_PASS = 16
MPOW_TUNE_FORCE = 1
TILE_TABLE_LEN = 17
MPOW_MAX_STEPS = 126
MPOW_NAIVE_MAX_P = 4096
MPOW_NOALLOC_MAX_N = 2048

MPOW_KERNEL_GEMM_F32_128 = 0
MPOW_KERNEL_GEMM_F32_64 = 1
MPOW_KERNEL_GEMM_F32_32 = 2
MPOW_KERNEL_GEMM_F16X3_128 = 3
MPOW_KERNEL_GEMM_BF16X3_128 = 4
MPOW_KERNEL_GEMM_F32_256 = 5
MPOW_KERNEL_GEMM_F32_128x64 = 6
MPOW_KERNEL_GEMM_F16X3_256 = 7
MPOW_KERNEL_GEMM_BF16X3_256 = 8
MPOW_KERNEL_GEMM_F32_32_K4 = 9
MPOW_KERNEL_GEMM_F32_32_K8 = 10
MPOW_KERNEL_GEMM_F32_64_K2 = 11
MPOW_KERNEL_GEMM_F32_128_K2 = 12
MPOW_KERNEL_GEMM_BF16X6_128 = 13
MPOW_KERNEL_GEMM_BF16X6_256 = 14
MPOW_KERNEL_GEMM_F32_64_DMA = 15
MPOW_KERNEL_GEMM_F32_128_DMA = 16
MPOW_KERNEL_GEMM_F32_256x128_DMA = 17
MPOW_KERNEL_GEMM_F32_32_K4_DMA = 18
MPOW_KERNEL_POWER_WG = 19
MPOW_KERNEL_GEMM_F32_32_K8_DMA = 20
MPOW_KERNEL_COUNT = 21

# every symbol include/mpow.h declares
EXPORTS = (
    "mpow_status_str", "mpow_gemm_count", "mpow_schedule", "mpow_window_schedule", "mpow_workspace_bytes",
    "mpow_plan_create", "mpow_plan_destroy", "mpow_run", "mpow_run_naive", "mpow_run_noalloc",
    "mpow_run_batched", "mpow_expm",
    "mpow_last_device_error", "mpow_plan_timing", "mpow_plan_timing_reset",
    "mpow_plan_tile_table", "mpow_plan_autotune", "mpow_plan_kernel_for", "mpow_plan_set_kernel",
    "mpow_fp32_kernel_for",
    "mpow_mode_for_tolerance",
    "mpow_srv_create", "mpow_srv_submit", "mpow_srv_poll", "mpow_srv_wait_idle", "mpow_srv_stats",
    "mpow_srv_destroy", "mpow_srv_simulate",
)

_lib = None


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("route", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_end", ctypes.c_double)]


class SrvStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("in_flight", ctypes.c_int32),
                ("arena_capacity", ctypes.c_size_t), ("arena_in_use", ctypes.c_size_t),
                ("arena_peak", ctypes.c_size_t), ("last_device_error", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SimConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("n_streams", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("batch_cap", ctypes.c_int32), ("pad", ctypes.c_int32), ("plain_flops", ctypes.c_double),
                ("batch_flops", ctypes.c_double), ("launch_overhead_s", ctypes.c_double)]


class SimRequest(ctypes.Structure):
    _fields_ = [("t_arrive", ctypes.c_double), ("n", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("p", ctypes.c_int64)]


class SimResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("route", ctypes.c_int32), ("stream", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_end", ctypes.c_double)]


class MpowError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {mpow_status_str(status)} (status {status})")
        self.status = status


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1204_3052_amd.build`")
    # One HIP runtime per process: when PyTorch is present, load its runtime
    # first so that the library's libamdhip64.so.7 dependency resolves to the
    # copy torch uses (a second runtime would not see the GPU).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    P = c.c_void_p
    sig = {
        "mpow_status_str": (c.c_char_p, [c.c_int]),
        "mpow_gemm_count": (c.c_int, [c.c_int64]),
        "mpow_fp32_kernel_for": (c.c_int, [c.c_int, c.c_int]),
        "mpow_schedule": (c.c_int, [c.c_int64, P, c.c_int]),
        "mpow_window_schedule": (c.c_int, [c.c_int64, c.c_int, P, c.c_int, c.POINTER(c.c_int)]),
        "mpow_workspace_bytes": (c.c_size_t, [c.c_int, c.c_int, c.c_int]),
        "mpow_plan_create": (c.c_int, [c.POINTER(P), c.c_int, c.c_int, c.c_int, c.c_int, c.c_uint32]),
        "mpow_plan_destroy": (c.c_int, [P]),
        "mpow_run": (c.c_int, [P, P, c.c_int, c.c_int64, P, P, P]),
        "mpow_run_naive": (c.c_int, [P, P, c.c_int, c.c_int64, P, P, P]),
        "mpow_run_noalloc": (c.c_int, [P, c.c_int, c.c_int64, P, P, P]),
        "mpow_expm": (c.c_int, [P, P, c.c_int, P, P, c.c_int, P]),
        "mpow_run_batched": (c.c_int, [P, c.c_int, P, P, P, P, P, P]),
        "mpow_last_device_error": (c.c_int, [P]),
        "mpow_plan_timing": (c.c_int, [P, c.c_int, c.POINTER(c.c_int64), c.POINTER(c.c_double),
                                       c.POINTER(c.c_double), c.POINTER(c.c_char_p)]),
        "mpow_plan_timing_reset": (c.c_int, [P]),
        "mpow_plan_tile_table": (c.c_int, [P, P, c.c_int, c.c_int]),
        "mpow_plan_autotune": (c.c_int, [P, c.c_char_p, c.c_uint32]),
        "mpow_plan_kernel_for": (c.c_int, [P, c.c_int, c.c_int]),
        "mpow_plan_set_kernel": (c.c_int, [P, c.c_int]),
        "mpow_mode_for_tolerance": (c.c_int, [c.c_double, c.c_double, c.c_int]),
        "mpow_srv_create": (c.c_int, [c.POINTER(P), c.c_int, c.c_int, c.c_size_t, c.c_int, c.c_int, c.c_uint32]),
        "mpow_srv_submit": (c.c_int, [P, P, c.c_int, c.c_int64, c.c_int, P, P, c.POINTER(c.c_uint64)]),
        "mpow_srv_poll": (c.c_int, [P, c.POINTER(Completion), c.c_int]),
        "mpow_srv_wait_idle": (c.c_int, [P, c.c_double]),
        "mpow_srv_stats": (c.c_int, [P, c.POINTER(SrvStats)]),
        "mpow_srv_destroy": (c.c_int, [P]),
        "mpow_srv_simulate": (c.c_int, [c.POINTER(SimConfig), c.POINTER(SimRequest), c.c_int,
                                        c.POINTER(SimResult), c.POINTER(c.c_size_t)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != MPOW_SUCCESS:
        raise MpowError(status, what)


# ---------------------------------------------------------------- raw ABI

def mpow_status_str(status: int) -> str:
    return _load().mpow_status_str(int(status)).decode()


def mpow_gemm_count(p: int) -> int:
    return int(_load().mpow_gemm_count(int(p)))


def mpow_fp32_kernel_for(n: int, aligned: bool = True) -> int:
    """The float32 product kernel id mpow_run uses at size n by default."""
    return int(_load().mpow_fp32_kernel_for(int(n), 1 if aligned else 0))


def mpow_schedule(p: int) -> list:
    ops = (ctypes.c_uint8 * MPOW_MAX_STEPS)()
    g = _load().mpow_schedule(int(p), ctypes.cast(ops, ctypes.c_void_p), MPOW_MAX_STEPS)
    if g < 0:
        raise MpowError(MPOW_ERR_INVALID, "mpow_schedule")
    return [int(ops[i]) for i in range(g)]


def mpow_window_schedule(p: int, w: int = 0):
    """(ops as a list of (dst, x, y) slot triples, result slot); w = 0: fewest products."""
    c = ctypes
    r = c.c_int(-1)
    g = _load().mpow_window_schedule(int(p), int(w), None, 0, c.byref(r))
    if g < 0:
        raise MpowError(MPOW_ERR_INVALID, "mpow_window_schedule")
    buf = (c.c_uint8 * max(3 * g, 1))()
    g = _load().mpow_window_schedule(int(p), int(w), c.cast(buf, c.c_void_p), g, c.byref(r))
    return [(buf[3 * k], buf[3 * k + 1], buf[3 * k + 2]) for k in range(g)], r.value


def mpow_workspace_bytes(max_n: int, max_batch: int = 0, mode: int = MPOW_FP32) -> int:
    return int(_load().mpow_workspace_bytes(int(max_n), int(max_batch), int(mode)))


def mpow_plan_create(device: int, max_n: int, max_batch: int = 0, mode: int = MPOW_FP32,
                     flags: int = 0) -> int:
    h = ctypes.c_void_p()
    st = _load().mpow_plan_create(ctypes.byref(h), int(device), int(max_n), int(max_batch),
                                  int(mode), int(flags))
    _check(st, "mpow_plan_create")
    return h.value


def mpow_plan_destroy(plan: int) -> None:
    _check(_load().mpow_plan_destroy(plan), "mpow_plan_destroy")


def mpow_run(plan: int, A: int, n: int, p: int, out: int, log2_scale: int | None,
             stream: int | None) -> None:
    st = _load().mpow_run(plan, A, int(n), int(p), out, log2_scale or None, stream or None)
    _check(st, "mpow_run")


def mpow_run_naive(plan: int, A: int, n: int, p: int, out: int, log2_scale: int | None,
                   stream: int | None) -> None:
    st = _load().mpow_run_naive(plan, A, int(n), int(p), out, log2_scale or None, stream or None)
    _check(st, "mpow_run_naive")


def mpow_run_noalloc(A: int, n: int, p: int, out: int, log2_scale: int | None,
                     stream: int | None) -> None:
    st = _load().mpow_run_noalloc(A, int(n), int(p), out, log2_scale or None, stream or None)
    _check(st, "mpow_run_noalloc")


def mpow_expm(plan: int, A: int, n: int, out: int, log2_scale: int | None, squarings: int,
              stream: int | None) -> None:
    st = _load().mpow_expm(plan, A, int(n), out, log2_scale or None, int(squarings), stream or None)
    _check(st, "mpow_expm")


class BatchArgs:
    """The host arrays of one batch (input pointers, sizes, powers, output
    pointers) marshalled once, for calling mpow_run_batched repeatedly on the
    same matrices without rebuilding them."""

    def __init__(self, A_ptrs, ns, ps, out_ptrs):
        c = ctypes
        self.count = count = len(ns)
        if not (len(A_ptrs) == len(ps) == len(out_ptrs) == count):
            raise ValueError("batch arrays differ in length")
        self.a = (c.c_void_p * count)(*A_ptrs)
        self.o = (c.c_void_p * count)(*out_ptrs)
        self.n = (c.c_int * count)(*[int(x) for x in ns])
        self.p = (c.c_int64 * count)(*[int(x) for x in ps])


def mpow_run_batched(plan: int, count: int, A_ptrs, ns=None, ps=None, out_ptrs=None,
                     log2_scale: int | None = None, stream: int | None = None) -> None:
    """A_ptrs is either the list of input pointers (then ns, ps and out_ptrs
    are the other lists) or a BatchArgs (ns, ps and out_ptrs unused)."""
    c = ctypes
    b = A_ptrs if isinstance(A_ptrs, BatchArgs) else BatchArgs(A_ptrs, ns, ps, out_ptrs)
    if count > b.count:
        raise ValueError("count exceeds the batch arrays")
    st = _load().mpow_run_batched(plan, int(count), c.cast(b.a, c.c_void_p), c.cast(b.n, c.c_void_p),
                                  c.cast(b.p, c.c_void_p), c.cast(b.o, c.c_void_p),
                                  log2_scale or None, stream or None)
    _check(st, "mpow_run_batched")


def mpow_last_device_error(plan: int) -> int:
    return int(_load().mpow_last_device_error(plan))


def mpow_plan_timing(plan: int, kernel: int):
    """(launches, total_ms, total_flop, kernel symbol name)"""
    c = ctypes
    l, m, f, nm = c.c_int64(), c.c_double(), c.c_double(), c.c_char_p()
    _check(_load().mpow_plan_timing(plan, int(kernel), c.byref(l), c.byref(m), c.byref(f), c.byref(nm)),
           "mpow_plan_timing")
    return l.value, m.value, f.value, (nm.value.decode() if nm.value else None)


def mpow_plan_kernel_for(plan: int, n: int, aligned: bool = True) -> int:
    """The product kernel id mpow_run on this plan uses at size n."""
    return int(_load().mpow_plan_kernel_for(plan, int(n), 1 if aligned else 0))


def mpow_plan_timing_reset(plan: int) -> None:
    _check(_load().mpow_plan_timing_reset(plan), "mpow_plan_timing_reset")


def mpow_mode_for_tolerance(tol: float, floor: float = 0.0, wide_range: bool = False) -> int:
    """Fastest mode whose stated bar max(ABS, FACTOR * floor) is <= tol; -1 if none."""
    return int(_load().mpow_mode_for_tolerance(float(tol), float(floor), 1 if wide_range else 0))


def mpow_plan_set_kernel(plan: int, kernel: int) -> None:
    """Forces the plain-path product kernel (-1: per-size default)."""
    _check(_load().mpow_plan_set_kernel(plan, int(kernel)), "mpow_plan_set_kernel")


def mpow_plan_tile_table(plan: int, table=None) -> list:
    """Returns the batched kernel's tile table; replaces it first if given."""
    buf = (ctypes.c_int * TILE_TABLE_LEN)()
    if table is not None:
        for i, v in enumerate(table):
            buf[i] = int(v)
        _check(_load().mpow_plan_tile_table(plan, ctypes.cast(buf, ctypes.c_void_p), TILE_TABLE_LEN, 1),
               "mpow_plan_tile_table")
    _check(_load().mpow_plan_tile_table(plan, ctypes.cast(buf, ctypes.c_void_p), TILE_TABLE_LEN, 0),
           "mpow_plan_tile_table")
    return [int(v) for v in buf]


def mpow_plan_autotune(plan: int, cache_path: str | None = None, flags: int = 0) -> None:
    _check(_load().mpow_plan_autotune(plan, cache_path.encode() if cache_path else None, int(flags)),
           "mpow_plan_autotune")


def mpow_srv_create(device: int, max_n: int, hbm_budget: int, n_streams: int = 4,
                    max_batch: int = 1024, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(_load().mpow_srv_create(ctypes.byref(h), int(device), int(max_n), int(hbm_budget),
                                   int(n_streams), int(max_batch), int(flags)), "mpow_srv_create")
    return h.value


def mpow_srv_submit(srv: int, A: int, n: int, p: int, mode: int, out: int,
                    log2_scale: int | None = None) -> int:
    rid = ctypes.c_uint64()
    _check(_load().mpow_srv_submit(srv, A, int(n), int(p), int(mode), out, log2_scale or None,
                                   ctypes.byref(rid)), "mpow_srv_submit")
    return rid.value


def mpow_srv_poll(srv: int, max_items: int = 4096) -> list:
    buf = (Completion * max_items)()
    k = _load().mpow_srv_poll(srv, buf, max_items)
    if k < 0:
        raise MpowError(MPOW_ERR_INVALID, "mpow_srv_poll")
    return [{"id": buf[i].id, "status": buf[i].status, "route": buf[i].route,
             "t_submit": buf[i].t_submit, "t_start": buf[i].t_start, "t_end": buf[i].t_end}
            for i in range(k)]


def mpow_srv_wait_idle(srv: int, timeout_s: float = 60.0) -> None:
    _check(_load().mpow_srv_wait_idle(srv, float(timeout_s)), "mpow_srv_wait_idle")


def mpow_srv_stats(srv: int) -> dict:
    st = SrvStats()
    _check(_load().mpow_srv_stats(srv, ctypes.byref(st)), "mpow_srv_stats")
    return {f: getattr(st, f) for f, _ in SrvStats._fields_ if f != "pad"}


def mpow_srv_destroy(srv: int) -> None:
    _check(_load().mpow_srv_destroy(srv), "mpow_srv_destroy")


def mpow_srv_simulate(requests, hbm_budget: int, n_streams: int = 4, depth: int = 2,
                      batch_cap: int = 1024, plain_flops: float = 1e14, batch_flops: float = 5e13,
                      launch_overhead_s: float = 1e-5):
    """requests: sequence of (t_arrive, n, p, mode), sorted by t_arrive.
    Returns (list of result dicts, peak arena bytes)."""
    count = len(requests)
    cfg = SimConfig(hbm_budget=int(hbm_budget), n_streams=n_streams, depth=depth, batch_cap=batch_cap,
                    pad=0, plain_flops=plain_flops, batch_flops=batch_flops,
                    launch_overhead_s=launch_overhead_s)
    reqs = (SimRequest * max(count, 1))()
    for i, (t, n, p, mode) in enumerate(requests):
        reqs[i] = SimRequest(float(t), int(n), int(mode), int(p))
    res = (SimResult * max(count, 1))()
    peak = ctypes.c_size_t()
    _check(_load().mpow_srv_simulate(ctypes.byref(cfg), reqs, count, res, ctypes.byref(peak)),
           "mpow_srv_simulate")
    out = [{"status": res[i].status, "route": res[i].route, "stream": res[i].stream,
            "t_admit": res[i].t_admit, "t_start": res[i].t_start, "t_end": res[i].t_end}
           for i in range(count)]
    return out, peak.value


# ---------------------------------------------------------------- torch helpers

class Plan:
    """Owns an mpow plan; usable as a context manager."""

    def __init__(self, max_n: int, max_batch: int = 0, mode: int = MPOW_FP32, flags: int = 0,
                 device: int | None = None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.max_n, self.max_batch, self.mode, self.flags = max_n, max_batch, mode, flags
        self.handle = mpow_plan_create(self.device, max_n, max_batch, mode, flags)

    def close(self):
        if self.handle:
            mpow_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_matrix(A):
    import torch
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float32 or not A.is_cuda:
        raise TypeError("A must be a float32 CUDA (HIP) tensor")
    if A.dim() != 2 or A.shape[0] != A.shape[1] or not A.is_contiguous():
        raise ValueError("A must be a contiguous square matrix")


def _stream_handle(device, stream):
    import torch
    st = torch.cuda.current_stream(device) if stream is None else stream
    return st.cuda_stream


def run(A, p: int, plan: Plan | None = None, out=None, return_scale: bool = False, stream=None,
        mode: int | None = None):
    """A^p of a square float32 device tensor (mpow_run).

    mode: the product arithmetic (MPOW_FP32, MPOW_FP16X3, MPOW_BF16X3,
    MPOW_BF16X6); None takes the plan's, or MPOW_FP32 for a temporary plan.
    A given plan must have been created for that mode.  Returns `out` (A^p
    rounded to float32), or (M, s) with A^p = M * 2^s when return_scale is
    true; s is a one-element float64 device tensor."""
    import torch
    _check_matrix(A)
    n = A.shape[0]
    own = plan is None
    if own:
        plan = Plan(n, mode=MPOW_FP32 if mode is None else int(mode), device=A.device.index)
    elif mode is not None and int(mode) != plan.mode:
        raise ValueError(f"plan was created for mode {plan.mode}, not {mode}")
    try:
        if out is None:
            out = torch.empty_like(A)
        scale = torch.empty(1, dtype=torch.float64, device=A.device) if return_scale else None
        mpow_run(plan.handle, A.data_ptr(), n, p, out.data_ptr(),
                 scale.data_ptr() if scale is not None else None, _stream_handle(A.device, stream))
        if own:
            torch.cuda.synchronize(A.device)
    finally:
        if own:
            plan.close()
    return (out, scale) if return_scale else out


def run_batched(As, ps, plan: Plan | None = None, outs=None, return_scale: bool = False,
                stream=None):
    """Independent powers As[i]^ps[i] in one persistent launch (mpow_run_batched).

    As: sequence of square float32 device tensors (n <= 256) on one device;
    ps: powers.  Returns the list of outputs, or (outputs, s) with s a
    float64 device tensor of one log2 scale per matrix when return_scale is
    true.  A given plan must be a float32 plan with max_batch >= len(As) and
    max_n >= the largest n."""
    import torch
    As = list(As)
    ps = [int(p) for p in ps]
    if len(ps) != len(As):
        raise ValueError("As and ps differ in length")
    for A in As:
        _check_matrix(A)
    count = len(As)
    if count == 0:
        return ([], None) if return_scale else []
    dev = As[0].device
    if any(A.device != dev for A in As):
        raise ValueError("all matrices must be on one device")
    ns = [A.shape[0] for A in As]
    if outs is None:
        outs = [torch.empty_like(A) for A in As]
    own = plan is None
    if own:
        plan = Plan(max(ns), max_batch=count, device=dev.index)
    try:
        scale = torch.empty(count, dtype=torch.float64, device=dev) if return_scale else None
        mpow_run_batched(plan.handle, count, [A.data_ptr() for A in As], ns, ps,
                         [o.data_ptr() for o in outs],
                         scale.data_ptr() if scale is not None else None, _stream_handle(dev, stream))
        if own:
            torch.cuda.synchronize(dev)
    finally:
        if own:
            plan.close()
    return (outs, scale) if return_scale else outs


class Server:
    """Request server over mpow_srv_* (continuous batching of independent powers).

    submit() queues A^p and returns the request id; the server keeps the
    request's tensors alive until poll() has returned its completion record.
    Usable as a context manager; close() drains every request first."""

    def __init__(self, max_n: int, hbm_budget: int, n_streams: int = 4, max_batch: int = 1024,
                 device: int | None = None):
        import torch
        self.device = torch.cuda.current_device() if device is None else int(device)
        self.handle = mpow_srv_create(self.device, max_n, hbm_budget, n_streams, max_batch)
        self._held = {}

    def submit(self, A, p: int, mode: int = MPOW_FP32, out=None, return_scale: bool = False):
        """Queues A^p.  Returns (id, out) or (id, out, s) with s a one-element
        float64 device tensor; both are valid once the request has completed."""
        import torch
        _check_matrix(A)
        if out is None:
            out = torch.empty_like(A)
        scale = torch.empty(1, dtype=torch.float64, device=A.device) if return_scale else None
        rid = mpow_srv_submit(self.handle, A.data_ptr(), A.shape[0], int(p), int(mode), out.data_ptr(),
                              scale.data_ptr() if scale is not None else None)
        self._held[rid] = (A, out, scale)
        return (rid, out, scale) if return_scale else (rid, out)

    def poll(self, max_items: int = 4096) -> list:
        done = mpow_srv_poll(self.handle, max_items)
        for c in done:
            self._held.pop(c["id"], None)
        return done

    def wait_idle(self, timeout_s: float = 60.0) -> None:
        mpow_srv_wait_idle(self.handle, timeout_s)

    def stats(self) -> dict:
        return mpow_srv_stats(self.handle)

    def close(self):
        if self.handle:
            mpow_srv_destroy(self.handle)
            self.handle = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
