"""GPU test of mpow_run_noalloc, the entry point that allocates nothing: its
workspace is a fixed device array inside the library.  It runs the kernels
mpow_run runs on a float32 plan with default kernels, so both must give the
same bits; two calls in a row (the second smaller, the array keeping the
first call's contents) must each match, and the calls must not take device
memory."""
import numpy as np
import pytest

from paper_1204_3052_amd import inputs, mpow

from gpu_util import check_against_oracle, run_gpu

pytestmark = pytest.mark.gpu


def run_noalloc(A_np, p, log_scale=True, out_is_input=False, stream=None):
    import torch
    n = A_np.shape[0]
    A = torch.from_numpy(np.ascontiguousarray(A_np, dtype=np.float32)).cuda()
    out = A if out_is_input else torch.full_like(A, float("nan"))
    s = torch.full((1,), -12345.0, dtype=torch.float64, device=A.device) if log_scale else None
    st = torch.cuda.current_stream() if stream is None else stream
    print(f"  [gpu] mpow_run_noalloc n={n} p={p} log={log_scale}", flush=True)
    mpow.mpow_run_noalloc(A.data_ptr(), n, p, out.data_ptr(), s.data_ptr() if s is not None else None,
                          st.cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (float(s.item()) if s is not None else None)


@pytest.fixture(scope="module")
def plan():
    import torch
    assert torch.cuda.is_available()
    mpow._load()
    h = mpow.mpow_plan_create(0, mpow.MPOW_NOALLOC_MAX_N, 0, mpow.MPOW_FP32, 0)
    yield h
    mpow.mpow_plan_destroy(h)


def test_noalloc_equals_mpow_run_two_calls(plan):
    # calls in a row on the library's array, each after a larger one (the
    # array keeps the previous call's contents), then the plan's results
    cases = [(1500, 1023), (300, 77), (2048, 17), (33, 1000), (1, 5)]
    mats = {n: inputs.gaussian(n, 700 + n) for n, _ in cases}
    got = [(run_noalloc(mats[n], p, log_scale=log), n, p, log)
           for log in (True, False) for n, p in cases]
    for (Mn, sn), n, p, log in got:
        Mr, sr = run_gpu(plan, mats[n], p, log_scale=log)
        assert np.array_equal(Mn, Mr) and sn == sr, (n, p, log)
    A = inputs.gaussian(300, 5)
    M, s = run_noalloc(A, 77)
    err, tol, _ = check_against_oracle(M, s, A, 77, seed=5)
    assert err <= tol, (err, tol)


def test_noalloc_edge_cases(plan):
    # p = 0 and 1, out aliasing A, a vanishing nilpotent power, all-ones 2^k
    A = inputs.gaussian(100, 3)
    for p in (0, 1, 2):
        Mn, sn = run_noalloc(A, p)
        Mr, sr = run_gpu(plan, A, p)
        assert np.array_equal(Mn, Mr) and sn == sr, p
    Mn, sn = run_noalloc(A, 55, out_is_input=True)
    Mr, sr = run_gpu(plan, A, 55)
    assert np.array_equal(Mn, Mr) and sn == sr
    M, s = run_noalloc(inputs.shift_matrix(64), 64)
    assert s == 0 and not np.any(M)
    M, s = run_noalloc(inputs.ones_matrix(256), 300)
    assert s == 8 * 300 and np.all(M == 2.0 ** -8)


def test_noalloc_rejects_and_allocates_nothing(plan):
    import torch
    n = mpow.MPOW_NOALLOC_MAX_N + 1
    A = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    out = torch.empty_like(A)
    with pytest.raises(mpow.MpowError) as ei:
        mpow.mpow_run_noalloc(A.data_ptr(), n, 3, out.data_ptr(), None, None)
    assert ei.value.status == mpow.MPOW_ERR_UNSUPPORTED
    del A, out
    # a stream of the current device is accepted; device memory in use does
    # not grow over calls once the library's module is loaded
    B = torch.from_numpy(inputs.gaussian(1024, 1)).cuda()
    o = torch.empty_like(B)
    side = torch.cuda.Stream()
    mpow.mpow_run_noalloc(B.data_ptr(), 1024, 100, o.data_ptr(), None, side.cuda_stream)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for p in (100, 1023, 5):
        mpow.mpow_run_noalloc(B.data_ptr(), 1024, p, o.data_ptr(), None, side.cuda_stream)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 >= free0, (free0, free1)
