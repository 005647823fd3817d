"""Inputs and outputs that start 4 bytes past a 16-byte boundary.

The C ABI asks for 4-byte alignment only.  Such a matrix, with n a multiple
of 4, takes the 4-byte load paths: the register-staged product tiles instead
of the LDS-DMA ones, the split pass's scalar loads, the batched kernel's
plain instance.  With the float32 tile pinned to the one the aligned input
gets (an LDS-DMA tile runs as its register-staged twin on an unaligned
input; left to itself the library may pick a K-split tile there, which adds
in another order), those paths add every output's products in the same order
as the 16-byte paths, so each result must equal the aligned run's bit for
bit, and nothing may be written outside the output matrix."""
import numpy as np
import pytest

from paper_1204_3052_amd import inputs, mpow

pytestmark = pytest.mark.gpu

MODES = {"fp32": mpow.MPOW_FP32, "fp16x3": mpow.MPOW_FP16X3, "bf16x3": mpow.MPOW_BF16X3,
         "bf16x6": mpow.MPOW_BF16X6}
GUARD = 8  # floats before and after each matrix


class Placed:
    """A at float offset `off_in` of a device buffer, its output at float
    offset `off_out` of another, NaN guards around both."""

    def __init__(self, A, off_in, off_out):
        import torch
        n = A.shape[0]
        self.n, self.off_in, self.off_out = n, off_in, off_out
        self.src = torch.full((n * n + 2 * GUARD,), np.nan, dtype=torch.float32, device="cuda")
        self.src[off_in:off_in + n * n] = torch.from_numpy(A.ravel()).cuda()
        self.dst = torch.full((n * n + 2 * GUARD,), np.nan, dtype=torch.float32, device="cuda")
        self.scale = torch.full((1,), -777.0, dtype=torch.float64, device="cuda")
        self.a = self.src.data_ptr() + 4 * off_in
        self.o = self.dst.data_ptr() + 4 * off_out

    def result(self):
        import torch
        torch.cuda.synchronize()
        n, off = self.n, self.off_out
        d = self.dst.cpu().numpy()
        assert np.all(np.isnan(d[:off])) and np.all(np.isnan(d[off + n * n:])), "write outside out"
        return d[off:off + n * n].reshape(n, n), float(self.scale.item())


def stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


@pytest.fixture(scope="module", params=list(MODES))
def mplan(request):
    mode = MODES[request.param]
    h = mpow.mpow_plan_create(0, 2048, 0, mode, 0)
    yield mode, h
    mpow.mpow_plan_destroy(h)


@pytest.mark.parametrize("n", [64, 512, 516, 1024, 2048])
def test_run_offset_pointers_bit_identical(mplan, n):
    mode, h = mplan
    A = inputs.gaussian(n, 90 + n)
    if mode == mpow.MPOW_FP32:
        mpow.mpow_plan_set_kernel(h, mpow.mpow_fp32_kernel_for(n, True))
    try:
        for p in (2, 17):
            res = []
            for off_in, off_out in ((GUARD, GUARD), (GUARD + 1, GUARD), (GUARD, GUARD + 3)):
                pl = Placed(A, off_in, off_out)
                print(f"  [gpu] mpow_run mode={mode} n={n} p={p} in+{off_in} out+{off_out}", flush=True)
                mpow.mpow_run(h, pl.a, n, p, pl.o, pl.scale.data_ptr(), stream())
                res.append(pl.result())
            for M, s in res[1:]:
                assert s == res[0][1] and np.array_equal(M, res[0][0]), (mode, n, p)
    finally:
        if mode == mpow.MPOW_FP32:
            mpow.mpow_plan_set_kernel(h, -1)


@pytest.mark.parametrize("n", [64, 1024])
def test_expm_offset_pointers_bit_identical(n):
    h = mpow.mpow_plan_create(0, n, 0, mpow.MPOW_FP32, mpow.MPOW_FLAG_EXPM)
    try:
        mpow.mpow_plan_set_kernel(h, mpow.mpow_fp32_kernel_for(n, True))
        A = inputs.gaussian(n, 95 + n)
        res = []
        for off_in, off_out in ((GUARD, GUARD), (GUARD + 1, GUARD + 1)):
            pl = Placed(A, off_in, off_out)
            print(f"  [gpu] mpow_expm n={n} in+{off_in} out+{off_out}", flush=True)
            mpow.mpow_expm(h, pl.a, n, pl.o, pl.scale.data_ptr(), -1, stream())
            res.append(pl.result())
        assert res[1][1] == res[0][1] and np.array_equal(res[1][0], res[0][0])
    finally:
        mpow.mpow_plan_destroy(h)


def test_window_offset_pointers_bit_identical():
    h = mpow.mpow_plan_create(0, 1024, 0, mpow.MPOW_FP32, mpow.MPOW_FLAG_WINDOW)
    try:
        mpow.mpow_plan_set_kernel(h, mpow.mpow_fp32_kernel_for(1024, True))
        A = inputs.gaussian(1024, 97)
        res = []
        for off_in, off_out in ((GUARD, GUARD), (GUARD + 1, GUARD + 2)):
            pl = Placed(A, off_in, off_out)
            print(f"  [gpu] mpow_run window n=1024 p=1023 in+{off_in} out+{off_out}", flush=True)
            mpow.mpow_run(h, pl.a, 1024, 1023, pl.o, pl.scale.data_ptr(), stream())
            res.append(pl.result())
        assert res[1][1] == res[0][1] and np.array_equal(res[1][0], res[0][0])
    finally:
        mpow.mpow_plan_destroy(h)


def test_batched_offset_pointer_bit_identical():
    # one matrix 4 bytes off a 16-byte boundary moves the whole batch off the
    # LDS-DMA instance; every result must stay what the aligned batch gives
    import torch
    ns = [16, 64, 100, 128, 256, 252]
    ps = [17, 100, 3, 1000, 17, 2]
    mats = [inputs.gaussian(n, 300 + i) for i, n in enumerate(ns)]
    h = mpow.mpow_plan_create(0, 256, len(ns), mpow.MPOW_FP32, 0)
    try:
        res = []
        for shift in (0, 1):
            places = [Placed(A, GUARD + (shift if i == 3 else 0), GUARD) for i, A in enumerate(mats)]
            scale = torch.full((len(ns),), -777.0, dtype=torch.float64, device="cuda")
            print(f"  [gpu] mpow_run_batched count={len(ns)} shift={shift}", flush=True)
            mpow.mpow_run_batched(h, len(ns), [pl.a for pl in places], ns, ps, [pl.o for pl in places],
                                  scale.data_ptr(), stream())
            torch.cuda.synchronize()
            sc = scale.cpu().numpy()
            res.append([(pl.result()[0], float(sc[i])) for i, pl in enumerate(places)])
        for (M0, s0), (M1, s1), n, p in zip(res[0], res[1], ns, ps):
            assert s0 == s1 and np.array_equal(M0, M1), (n, p)
    finally:
        mpow.mpow_plan_destroy(h)
