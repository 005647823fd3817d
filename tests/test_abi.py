"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, rejects bad arguments before touching a
device, and its exponent schedule agrees with the oracle's."""
import ctypes
import os
import re

import pytest

import oracle
from paper_1204_3052_amd import mpow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpow.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mpow.LIB_PATH):
        from paper_1204_3052_amd import build
        build.build(verbose=False)
    return mpow._load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpow_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert header_functions() == sorted(mpow.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(mpow.LIB_PATH)
    for name in header_functions():
        assert hasattr(raw, name), name


def test_status_strings(lib):
    for code in range(7):
        assert isinstance(mpow.mpow_status_str(code), str)
    assert mpow.mpow_status_str(99) == "unknown status"


@pytest.mark.parametrize("p", list(range(0, 200)) + [1000, 1023, 2 ** 20 - 1, 2 ** 20, 2 ** 62 + 5, 2 ** 63 - 1])
def test_schedule_matches_oracle(lib, p):
    ops = mpow.mpow_schedule(p)
    assert ["S" if o == 0 else "M" for o in ops] == oracle.schedule(p)
    assert mpow.mpow_gemm_count(p) == len(ops) == oracle.gemm_count(p)


def test_schedule_rejects(lib):
    assert lib.mpow_gemm_count(-1) == -1
    assert lib.mpow_schedule(-5, None, 10) == -1
    assert lib.mpow_schedule(17, None, 10) == -1   # ops NULL while G(17)=5 > 0
    buf = (ctypes.c_uint8 * 4)()
    assert lib.mpow_schedule(17, ctypes.cast(buf, ctypes.c_void_p), 4) == -1  # cap too small
    assert lib.mpow_schedule(1, None, 0) == 0
    assert lib.mpow_gemm_count(2 ** 63 - 1) == 124 <= mpow.MPOW_MAX_STEPS


def test_workspace_bytes(lib):
    assert mpow.mpow_workspace_bytes(0) == 0
    assert mpow.mpow_workspace_bytes(16, -1) == 0
    assert mpow.mpow_workspace_bytes(16, 0, 9) == 0
    b = mpow.mpow_workspace_bytes(8192)
    assert 2 * 8192 * 8192 * 4 <= b < 2 * 8192 * 8192 * 4 + 8 * 2 ** 20


def test_null_arguments_rejected_without_device(lib):
    P = ctypes.c_void_p
    assert lib.mpow_plan_create(None, 0, 16, 0, 0, 0) == mpow.MPOW_ERR_INVALID
    h = P()
    assert lib.mpow_plan_create(ctypes.byref(h), 0, 0, 0, 0, 0) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_create(ctypes.byref(h), 0, 16, -1, 0, 0) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_create(ctypes.byref(h), 0, 16, 0, 7, 0) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_create(ctypes.byref(h), 0, 16, 0, 0, 1 << 10) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_run(None, 16, 4, 3, 16, None, None) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_run_batched(None, 1, None, None, None, None, None, None) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_timing(None, 0, None, None, None, None) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_timing_reset(None) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_set_kernel(None, -1) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_plan_destroy(None) == mpow.MPOW_SUCCESS
    assert lib.mpow_last_device_error(None) == 0


def test_noalloc_rejects_without_device(lib):
    # argument errors and sizes beyond the fixed workspace are reported before
    # any device call (the pointers below are never dereferenced)
    f = lib.mpow_run_noalloc
    A, out = 1 << 20, 1 << 30
    assert f(None, 16, 3, out, None, None) == mpow.MPOW_ERR_INVALID
    assert f(A, 0, 3, out, None, None) == mpow.MPOW_ERR_INVALID
    assert f(A, 16, -1, out, None, None) == mpow.MPOW_ERR_INVALID
    assert f(A + 2, 16, 3, out, None, None) == mpow.MPOW_ERR_INVALID
    assert f(A, 16, 3, A + 4, None, None) == mpow.MPOW_ERR_INVALID
    n = mpow.MPOW_NOALLOC_MAX_N + 1
    assert f(A, n, 3, A + 4 * n * n, None, None) == mpow.MPOW_ERR_UNSUPPORTED
    assert mpow.MPOW_NOALLOC_MAX_N == 2048


def test_plan_create_without_gpu_reports_device_error(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    st = lib.mpow_plan_create(ctypes.byref(h), 0, 64, 0, 0, 0)
    assert st == mpow.MPOW_ERR_DEVICE and not h.value


def test_tolerance_modes_match_library():
    from oracle import tolerance
    assert (tolerance.MODE_FP32, tolerance.MODE_FP16X3, tolerance.MODE_BF16X3, tolerance.MODE_BF16X6) == \
        (mpow.MPOW_FP32, mpow.MPOW_FP16X3, mpow.MPOW_BF16X3, mpow.MPOW_BF16X6)
    assert tolerance.tol_mode(mpow.MPOW_BF16X6, 0.0) == 1e-5
    assert tolerance.tol_fp32(0.0) == 1e-5 and tolerance.tol_fp32(1e-3) == 64e-3
    assert tolerance.tol_mode(mpow.MPOW_BF16X3, 0.0) == 2e-4
    assert tolerance.tol_expm(0.0, 0) == 1e-5 and tolerance.tol_expm(0.0, 10) == 4 * 2.0 ** -14


def test_mode_for_tolerance(lib):
    M = mpow
    assert M.mpow_mode_for_tolerance(1e-3) == M.MPOW_BF16X3
    assert M.mpow_mode_for_tolerance(2e-4) == M.MPOW_BF16X3
    assert M.mpow_mode_for_tolerance(1e-4) == M.MPOW_FP16X3
    assert M.mpow_mode_for_tolerance(1e-4, wide_range=True) == M.MPOW_BF16X6
    assert M.mpow_mode_for_tolerance(1e-5) == M.MPOW_FP16X3
    assert M.mpow_mode_for_tolerance(9e-6) == -1
    assert M.mpow_mode_for_tolerance(float("nan")) == -1
    assert M.mpow_mode_for_tolerance(1e-3, -1.0) == -1
    # an ill-conditioned power: the floor term decides
    assert M.mpow_mode_for_tolerance(5e-4, 1e-6) == M.MPOW_FP16X3
    assert M.mpow_mode_for_tolerance(5e-5, 1e-6) == -1


@pytest.mark.parametrize("floor", [0.0, 1e-9, 3e-7, 1e-6, 2e-5, 1e-3])
@pytest.mark.parametrize("tol", [1e-6, 1e-5, 3e-5, 1e-4, 2e-4, 1e-3, 1e-2, 0.5])
def test_mode_for_tolerance_meets_the_stated_bars(lib, tol, floor):
    # the chosen mode's bar (oracle/tolerance.py, the bars the tests enforce)
    # is within tol, and no faster mode's bar is
    from oracle import tolerance
    speed_order = [mpow.MPOW_BF16X3, mpow.MPOW_FP16X3, mpow.MPOW_BF16X6, mpow.MPOW_FP32]
    for wide in (False, True):
        m = mpow.mpow_mode_for_tolerance(tol, floor, wide)
        ok = [x for x in speed_order if tolerance.tol_mode(x, floor) <= tol
              and not (wide and x == mpow.MPOW_FP16X3)]
        assert m == (ok[0] if ok else -1), (tol, floor, wide, m, ok)


def test_expm_rejects_without_device(lib):
    assert lib.mpow_expm(None, 16, 4, 32, None, -1, None) == mpow.MPOW_ERR_INVALID


def replay_exponents(ops, result):
    """Exponent of A held by every slot after the products (A = 1)."""
    e = {0: 1}
    for dst, x, y in ops:
        assert x in e and y in e, (dst, x, y)  # operands written before use
        e[dst] = e[x] + e[y]
    return e[result]


@pytest.mark.parametrize("p", list(range(1, 300)) + [1000, 1023, 4095, 12345, 2 ** 20 - 1, 2 ** 20,
                                                      2 ** 62 + 5, 2 ** 63 - 1])
def test_window_schedule_reaches_p(lib, p):
    counts = {}
    for w in (1, 2, 3):
        ops, r = mpow.mpow_window_schedule(p, w)
        assert replay_exponents(ops, r) == p, (p, w)
        assert all(s < 7 for op in ops for s in op)
        counts[w] = len(ops)
    assert counts[1] == mpow.mpow_gemm_count(p)  # w = 1 is the binary schedule
    ops, r = mpow.mpow_window_schedule(p, 0)
    assert replay_exponents(ops, r) == p
    assert len(ops) == min(counts.values())


def test_window_schedule_counts_and_rejects(lib):
    assert len(mpow.mpow_window_schedule(2 ** 20 - 1, 3)[0]) == 27
    assert len(mpow.mpow_window_schedule(1023, 0)[0]) == 14
    assert mpow.mpow_window_schedule(1, 0) == ([], 0)
    r = ctypes.c_int()
    assert lib.mpow_window_schedule(0, 0, None, 0, ctypes.byref(r)) == -1
    assert lib.mpow_window_schedule(5, 4, None, 0, ctypes.byref(r)) == -1
    assert lib.mpow_window_schedule(5, 1, None, 0, None) == -1
    buf = (ctypes.c_uint8 * 3)()
    assert lib.mpow_window_schedule(1023, 1, ctypes.cast(buf, ctypes.c_void_p), 1, ctypes.byref(r)) == -1


def test_fp32_kernel_for_default_choice():
    # Host-side default product kernel per size: K-split tiles below 768, then
    # the LDS-DMA tile whose tile count best fills whole waves of 256 CUs
    # (16-byte loads), the register-staged tiles otherwise.
    k = mpow.mpow_fp32_kernel_for
    assert k(0) == -1 and k(-5) == -1
    assert k(4) == k(300) == k(512) == mpow.MPOW_KERNEL_GEMM_F32_32_K8_DMA
    assert k(1) == k(513) == k(516) == k(767) == mpow.MPOW_KERNEL_GEMM_F32_32_K4
    assert k(300, False) == mpow.MPOW_KERNEL_GEMM_F32_32_K4
    assert k(768) == k(1024) == k(1536) == k(3072) == mpow.MPOW_KERNEL_GEMM_F32_64_DMA
    assert k(2048) == k(6144) == mpow.MPOW_KERNEL_GEMM_F32_128_DMA
    assert k(2600) == k(4096) == k(8192) == mpow.MPOW_KERNEL_GEMM_F32_256x128_DMA
    # beyond a 32-bit buffer range: the register-staged 256 x 256 tile
    assert k(23170) != mpow.MPOW_KERNEL_GEMM_F32_256 and k(23172) == mpow.MPOW_KERNEL_GEMM_F32_256
    # no 16-byte loads: same-order or K-split register-staged tiles
    assert k(1000, False) == mpow.MPOW_KERNEL_GEMM_F32_64_K2
    assert k(2048, False) == mpow.MPOW_KERNEL_GEMM_F32_128_K2
    assert k(3000, False) == mpow.MPOW_KERNEL_GEMM_F32_64
    assert k(8192, False) == mpow.MPOW_KERNEL_GEMM_F32_128
