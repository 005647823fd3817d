"""GPU parity of the split-precision modes (FP16X3, BF16X3, BF16X6) against
the FP64 oracle, through the C ABI.  FP16X3 and BF16X6 must meet the float32
tolerance; BF16X3 its own looser stated tolerance.  0/1 and power-of-two
structure is exact in all (the lower parts are zero), as are small
integers."""
import numpy as np
import pytest

import oracle
from paper_1204_3052_amd import inputs, mpow

from gpu_util import run_gpu, tol_mode

pytestmark = pytest.mark.gpu

MODES = {"fp16x3": mpow.MPOW_FP16X3, "bf16x3": mpow.MPOW_BF16X3, "bf16x6": mpow.MPOW_BF16X6}


@pytest.fixture(scope="module", params=list(MODES))
def mplan(request):
    mode = MODES[request.param]
    h = mpow.mpow_plan_create(0, 4096, 0, mode, 0)
    yield mode, h
    mpow.mpow_plan_destroy(h)


def check(mode, h, A, p, seed):
    M, s = run_gpu(h, A, p)
    ref = oracle.mpow_binary(A, p)
    err = oracle.rel_err(M, s, *ref)
    floor = oracle.floor_estimate(A, p, inputs.relative_signs(A.shape[0], 2000 + seed), ref=ref)
    tol = tol_mode(mode, floor)
    print(f"    mode={mode} n={A.shape[0]} p={p} err={err:.3e} tol={tol:.3e} floor={floor:.3e}")
    assert err <= tol, (mode, A.shape[0], p, err, tol)
    return err


@pytest.mark.parametrize("n", [1, 2, 17, 33, 100, 128, 129, 300, 513, 1030])
def test_split_parity_ragged(mplan, n):
    mode, h = mplan
    A = inputs.gaussian(n, 300 + n)
    for p in (2, 3, 17, 100):
        check(mode, h, A, p, n)


def test_split_p0_p1(mplan):
    mode, h = mplan
    A = inputs.gaussian(65, 1)
    M, s = run_gpu(h, A, 0)
    assert s == 0 and np.array_equal(M, np.eye(65, dtype=np.float32))
    out, _ = run_gpu(h, A, 1, log_scale=False)
    assert np.array_equal(out, A)


def test_split_n4096_p64_p1000(mplan):
    # N = 4096, N(0,1)/sqrt(N) entries, p in {64, 1000}.
    mode, h = mplan
    A = inputs.gaussian(4096, 4)
    for p in (64, 1000):
        check(mode, h, A, p, p)


def test_split_row_stochastic(mplan):
    mode, h = mplan
    A = inputs.row_stochastic(128, 0)
    err = check(mode, h, A, 64, 0)
    if mode == mpow.MPOW_FP16X3:
        assert err <= 1e-5


@pytest.mark.parametrize("n", [7, 64, 1000, 4096])
def test_split_permutation_exact(mplan, n):
    mode, h = mplan
    sigma = inputs.permutation_perm(n, n + 1)
    P = inputs.permutation_matrix(sigma)
    for p in (2, 17, 1023):
        tau, base, e = np.arange(n), sigma.copy(), p
        while e:
            if e & 1:
                tau = base[tau]
            base = base[base]
            e >>= 1
        M, s = run_gpu(h, P, p)
        assert np.array_equal(oracle.to_value(M, s), inputs.permutation_matrix(tau).astype(np.float64)), (n, p)


@pytest.mark.parametrize("k", [3, 7, 12])
def test_split_all_ones_exact(mplan, k):
    mode, h = mplan
    n = 2 ** k
    for p in (2, 17, 1000):
        M, s = run_gpu(h, inputs.ones_matrix(n), p)
        assert s == k * p and np.array_equal(M, np.full((n, n), 2.0 ** -k, np.float32)), (n, p, s)


def test_split_small_integers_exact(mplan):
    # Fibonacci block powers with every entry below 2^8: exact in both halves.
    mode, h = mplan
    F = [0, 1]
    while len(F) < 20:
        F.append(F[-1] + F[-2])
    A = inputs.fibonacci_blocks(6)
    for p in (1, 2, 5, 9, 12):
        M, s = run_gpu(h, A, p)
        V = oracle.to_value(M, s)
        assert V[0, 0] == F[p + 1] and V[0, 1] == F[p] and V[1, 1] == F[p - 1], p


def test_split_nilpotent(mplan):
    mode, h = mplan
    J = inputs.shift_matrix(40)
    M, s = run_gpu(h, J, 40)
    assert s == 0 and not np.any(M)
    M, s = run_gpu(h, J, 39)
    assert np.array_equal(oracle.to_value(M, s), np.eye(40, k=39))


def test_split_deterministic(mplan):
    mode, h = mplan
    A = inputs.gaussian(700, 8)
    M1, s1 = run_gpu(h, A, 33)
    M2, s2 = run_gpu(h, A, 33)
    assert np.array_equal(M1, M2) and s1 == s2


def test_split_input_scaling_exact(mplan):
    mode, h = mplan
    A = inputs.gaussian(150, 3)
    for k in (-80, 80):
        Ak = np.ldexp(A, k).astype(np.float32)
        M0, s0 = run_gpu(h, A, 17)
        M1, s1 = run_gpu(h, Ak, 17)
        assert np.array_equal(M0, M1) and s1 == s0 + 17 * k


def embed(A, m):
    """diag(A, 0) of size m: its powers are diag(A^p, 0) and its Frobenius
    norm is A's, so every scale matches A's run."""
    B = np.zeros((m, m), np.float32)
    B[:A.shape[0], :A.shape[0]] = A
    return B


def test_split_tile_kernels_bit_identical(mplan):
    # n = 1030 runs on 128 x 128 tiles and n = 4096 on 256 x 256 tiles (the
    # library's default picks); both add each output's products in the same
    # order, and the extra K range of the embedding contributes exact zeros.
    mode, h = mplan
    A = inputs.gaussian(1030, 41)
    for p in (2, 17):
        M0, s0 = run_gpu(h, A, p)
        M1, s1 = run_gpu(h, embed(A, 4096), p)
        assert s0 == s1
        assert np.array_equal(M1[:1030, :1030], M0)
        assert not np.any(M1[1030:, :]) and not np.any(M1[:, 1030:])


def test_split_parity_large_ragged(mplan):
    mode, h = mplan
    A = inputs.gaussian(2100, 42)
    for p in (3, 17):
        check(mode, h, A, p, p)


@pytest.mark.parametrize("n,p,tol,wide", [(512, 17, 3e-4, False), (512, 17, 3e-5, False),
                                          (300, 100, 1e-3, True), (300, 100, 1e-4, True)])
def test_mode_for_tolerance_end_to_end(n, p, tol, wide):
    # the mode picked for a requested tolerance (with the oracle's floor of
    # this input) meets that tolerance on the GPU
    A = inputs.gaussian(n, 60 + n)
    ref = oracle.mpow_binary(A, p)
    floor = oracle.floor_estimate(A, p, inputs.relative_signs(n, 61 + n), ref=ref)
    mode = mpow.mpow_mode_for_tolerance(tol, floor, wide)
    assert mode >= 0
    h = mpow.mpow_plan_create(0, n, 0, mode, 0)
    try:
        M, s = run_gpu(h, A, p)
    finally:
        mpow.mpow_plan_destroy(h)
    err = oracle.rel_err(M, s, *ref)
    print(f"    tol={tol} floor={floor:.2e} mode={mode} err={err:.3e}")
    assert err <= tol


BF16_KERNELS = {mpow.MPOW_BF16X3: (mpow.MPOW_KERNEL_GEMM_BF16X3_128, mpow.MPOW_KERNEL_GEMM_BF16X3_256),
                mpow.MPOW_BF16X6: (mpow.MPOW_KERNEL_GEMM_BF16X6_128, mpow.MPOW_KERNEL_GEMM_BF16X6_256)}


@pytest.mark.parametrize("mode", [mpow.MPOW_BF16X3, mpow.MPOW_BF16X6])
def test_fused_split_equals_split_pass(mode):
    # The BF16 products write the next operand's parts in their epilogue
    # (parts of the unnormalised result, the exponent folded into the next
    # product); the separate pass splits the normalised float32 result.  BF16
    # rounding commutes with exact power-of-two scaling, so both give the same
    # bits.  The fused plan's workspace starts NaN-filled: only what the
    # products write may be read.
    fused = mpow.mpow_plan_create(0, 1100, 0, mode, mpow.MPOW_FLAG_POISON)
    ref = mpow.mpow_plan_create(0, 1100, 0, mode, mpow.MPOW_FLAG_SPLIT_PASS)
    try:
        for kernel in (-1,) + BF16_KERNELS[mode]:
            mpow.mpow_plan_set_kernel(fused, kernel)
            mpow.mpow_plan_set_kernel(ref, kernel)
            for n in (1, 17, 100, 129, 300, 1030):
                A = inputs.gaussian(n, 4000 + n)
                for p in (2, 3, 17, 100):
                    for log in (True, False):
                        Mf, sf = run_gpu(fused, A, p, log_scale=log)
                        Mr, sr = run_gpu(ref, A, p, log_scale=log)
                        assert np.array_equal(Mf, Mr) and sf == sr, (kernel, n, p, log)
            # an input scaled far from 1: the parts of the first product's
            # result come from the exactly rescaled values
            A = np.ldexp(inputs.gaussian(256, 9), 90).astype(np.float32)
            Mf, sf = run_gpu(fused, A, 77)
            Mr, sr = run_gpu(ref, A, 77)
            assert np.array_equal(Mf, Mr) and sf == sr, kernel
    finally:
        mpow.mpow_plan_destroy(fused)
        mpow.mpow_plan_destroy(ref)
