"""Every product kernel, forced through mpow_plan_set_kernel, on ragged
sizes: the float32 kernels without a K split agree bit for bit (they add each
output's products in the same order), the K-split kernels are deterministic
and meet the float32 tolerance against the FP64 oracle, and the two tile
sizes of each split-precision mode agree bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1204_3052_amd import inputs, mpow

from gpu_util import check_against_oracle, run_gpu, tol_mode

pytestmark = pytest.mark.gpu

DMA = [mpow.MPOW_KERNEL_GEMM_F32_256, mpow.MPOW_KERNEL_GEMM_F32_64_DMA, mpow.MPOW_KERNEL_GEMM_F32_128_DMA,
       mpow.MPOW_KERNEL_GEMM_F32_256x128_DMA]
SAME_ORDER = [mpow.MPOW_KERNEL_GEMM_F32_128, mpow.MPOW_KERNEL_GEMM_F32_64, mpow.MPOW_KERNEL_GEMM_F32_32,
              mpow.MPOW_KERNEL_GEMM_F32_128x64] + DMA
K_SPLIT = [mpow.MPOW_KERNEL_GEMM_F32_32_K4, mpow.MPOW_KERNEL_GEMM_F32_32_K8,
           mpow.MPOW_KERNEL_GEMM_F32_64_K2, mpow.MPOW_KERNEL_GEMM_F32_128_K2,
           mpow.MPOW_KERNEL_GEMM_F32_32_K4_DMA, mpow.MPOW_KERNEL_GEMM_F32_32_K8_DMA]
# the LDS-DMA tiles run where n % 4 == 0 (100, 300, 700, 1028), the others
# fall back to a same-order tile
SIZES = [1, 33, 100, 257, 300, 513, 700, 1028, 1030]


@pytest.fixture(scope="module")
def fplan():
    h = mpow.mpow_plan_create(0, 1100, 0, mpow.MPOW_FP32, 0)
    yield h
    mpow.mpow_plan_destroy(h)


def forced(h, kernel, A, p):
    mpow.mpow_plan_set_kernel(h, kernel)
    try:
        return run_gpu(h, A, p)
    finally:
        mpow.mpow_plan_set_kernel(h, -1)


@pytest.mark.parametrize("n", SIZES)
def test_same_order_kernels_bit_identical(fplan, n):
    A = inputs.gaussian(n, 700 + n)
    for p in (2, 17):
        runs = [forced(fplan, k, A, p) for k in SAME_ORDER]
        M0, s0 = runs[0]
        for k, (M, s) in zip(SAME_ORDER[1:], runs[1:]):
            assert s == s0 and np.array_equal(M, M0), (n, p, k)
        err, tol, _ = check_against_oracle(M0, s0, A, p, seed=n)
        assert err <= tol, (n, p, err, tol)


@pytest.mark.parametrize("kernel", DMA)
@pytest.mark.parametrize("n", [300, 1028])
def test_dma_tile_operand_scale_paths(fplan, kernel, n):
    # The LDS-DMA tiles apply the operand scales 2^-eX, 2^-eY to their sums
    # when eX + eY keeps the unscaled product in the normal range, else to the
    # operands.  Inputs scaled by 2^k (exact) push the first product onto the
    # second path: M must be bit-identical to the unscaled run's, s shifted by
    # exactly k p, and both must equal the 128 x 128 tile's bits.
    A = inputs.gaussian(n, 900 + n)
    for p in (2, 17):
        M0, s0 = forced(fplan, kernel, A, p)
        for k in (70, -40, -70):
            Ak = np.ldexp(A, k).astype(np.float32)
            assert np.array_equal(np.ldexp(Ak, -k), A)
            M, s = forced(fplan, kernel, Ak, p)
            assert s == s0 + k * p and np.array_equal(M, M0), (n, p, k)
            M1, s1 = forced(fplan, mpow.MPOW_KERNEL_GEMM_F32_128, Ak, p)
            assert s1 == s and np.array_equal(M1, M), (n, p, k)


@pytest.mark.parametrize("ks", [4, 8])
@pytest.mark.parametrize("n", [4, 36, 100, 300, 508, 512])
def test_k4_whole_k_tile_equals_k4(fplan, n, ks):
    # The 32 x 32 tile with a 4- or 8-way K split and the whole K range in
    # LDS adds in the register-staged K-split tile's order: the same bits,
    # also where an input's scale sends the first product down the
    # operand-scaled path.
    reg, dma = {4: (mpow.MPOW_KERNEL_GEMM_F32_32_K4, mpow.MPOW_KERNEL_GEMM_F32_32_K4_DMA),
                8: (mpow.MPOW_KERNEL_GEMM_F32_32_K8, mpow.MPOW_KERNEL_GEMM_F32_32_K8_DMA)}[ks]
    A = inputs.gaussian(n, 1300 + n)
    for p in (2, 17, 100):
        for k in (0, 70, -70):
            Ak = np.ldexp(A, k).astype(np.float32)
            M0, s0 = forced(fplan, reg, Ak, p)
            M1, s1 = forced(fplan, dma, Ak, p)
            assert s0 == s1 and np.array_equal(M0, M1), (n, p, k)
            if k == 0:
                err, tol, _ = check_against_oracle(M1, s1, A, p, seed=n)
                assert err <= tol, (n, p, err, tol)


@pytest.mark.parametrize("kernel", K_SPLIT)
@pytest.mark.parametrize("n", SIZES)
def test_k_split_kernels_parity_and_deterministic(fplan, kernel, n):
    A = inputs.gaussian(n, 700 + n)
    for p in (2, 17, 100):
        M, s = forced(fplan, kernel, A, p)
        M2, s2 = forced(fplan, kernel, A, p)
        assert s2 == s and np.array_equal(M2, M)
        err, tol, floor = check_against_oracle(M, s, A, p, seed=n)
        print(f"    kernel={kernel} n={n} p={p} err={err:.3e} tol={tol:.3e}")
        assert err <= tol, (kernel, n, p, err, tol)


@pytest.mark.parametrize("kernel", K_SPLIT)
def test_k_split_exact_cases(fplan, kernel):
    # 0/1 and small-integer results are exact in any summation order
    sigma = inputs.permutation_perm(300, 5)
    tau = np.arange(300)
    for _ in range(97):  # sigma^97 as an index map, one composition at a time
        tau = sigma[tau]
    M, s = forced(fplan, kernel, inputs.permutation_matrix(sigma), 97)
    assert np.array_equal(oracle.to_value(M, s), inputs.permutation_matrix(tau).astype(np.float64))
    J = np.ones((64, 64), np.float32)
    M, s = forced(fplan, kernel, J, 9)
    assert np.array_equal(oracle.to_value(M, s), np.full((64, 64), 64.0 ** 8))


@pytest.mark.parametrize("mode,kernels", [
    (mpow.MPOW_FP16X3, [mpow.MPOW_KERNEL_GEMM_F16X3_128, mpow.MPOW_KERNEL_GEMM_F16X3_256]),
    (mpow.MPOW_BF16X3, [mpow.MPOW_KERNEL_GEMM_BF16X3_128, mpow.MPOW_KERNEL_GEMM_BF16X3_256]),
    (mpow.MPOW_BF16X6, [mpow.MPOW_KERNEL_GEMM_BF16X6_128, mpow.MPOW_KERNEL_GEMM_BF16X6_256]),
])
def test_split_mode_tile_sizes_bit_identical(mode, kernels):
    h = mpow.mpow_plan_create(0, 1100, 0, mode, 0)
    try:
        # n = 17 and 40 give the multi-stage kernels fewer K tiles than (or
        # as many as) they have LDS stages
        for n in (17, 40, 100, 513, 1030):
            A = inputs.gaussian(n, 800 + n)
            for p in (3, 17):
                (M0, s0), (M1, s1) = [forced(h, k, A, p) for k in kernels]
                assert s0 == s1 and np.array_equal(M0, M1), (mode, n, p)
                ref = oracle.mpow_binary(A, p)
                err = oracle.rel_err(M0, s0, *ref)
                floor = oracle.floor_estimate(A, p, inputs.relative_signs(n, 900 + n), ref=ref)
                assert err <= tol_mode(mode, floor), (mode, n, p, err)
    finally:
        mpow.mpow_plan_destroy(h)


def test_set_kernel_rejects_other_modes():
    h = mpow.mpow_plan_create(0, 64, 0, mpow.MPOW_FP32, 0)
    try:
        for bad in (-2, mpow.MPOW_KERNEL_GEMM_F16X3_128, mpow.MPOW_KERNEL_GEMM_BF16X3_256,
                    mpow.MPOW_KERNEL_GEMM_BF16X6_128, mpow.MPOW_KERNEL_COUNT, 99):
            with pytest.raises(mpow.MpowError):
                mpow.mpow_plan_set_kernel(h, bad)
    finally:
        mpow.mpow_plan_destroy(h)
    h = mpow.mpow_plan_create(0, 64, 0, mpow.MPOW_FP16X3, 0)
    try:
        for bad in (mpow.MPOW_KERNEL_GEMM_F32_128, mpow.MPOW_KERNEL_GEMM_BF16X3_128,
                    mpow.MPOW_KERNEL_GEMM_BF16X6_128):
            with pytest.raises(mpow.MpowError):
                mpow.mpow_plan_set_kernel(h, bad)
        mpow.mpow_plan_set_kernel(h, mpow.MPOW_KERNEL_GEMM_F16X3_256)
        mpow.mpow_plan_set_kernel(h, -1)
    finally:
        mpow.mpow_plan_destroy(h)
