"""GPU tests of the whole-power workgroup kernel on the single-matrix path
(mpow_run with MPOW_KERNEL_POWER_WG forced, n <= 128): one launch of one
workgroup that keeps its operands in LDS.  It accumulates every product in
the order of the float32 tiles without a K split, so it must give their bits;
it must also meet the oracle's bar and the exact structural results."""
import numpy as np
import pytest

import oracle
from paper_1204_3052_amd import inputs, mpow

from gpu_util import check_against_oracle, run_gpu

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 5, 16, 17, 31, 32, 33, 63, 64, 65, 96, 100, 127, 128]
POWERS = [0, 1, 2, 3, 17, 100, 1000]


@pytest.fixture(scope="module")
def wplans():
    import torch
    assert torch.cuda.is_available()
    mpow._load()
    hw = mpow.mpow_plan_create(0, 256, 0, mpow.MPOW_FP32, 0)
    mpow.mpow_plan_set_kernel(hw, mpow.MPOW_KERNEL_POWER_WG)
    hs = mpow.mpow_plan_create(0, 256, 0, mpow.MPOW_FP32, 0)
    mpow.mpow_plan_set_kernel(hs, mpow.MPOW_KERNEL_GEMM_F32_64)
    yield hw, hs
    mpow.mpow_plan_destroy(hw)
    mpow.mpow_plan_destroy(hs)


@pytest.mark.parametrize("n", SIZES)
def test_power_wg_equals_same_order_tiles(wplans, n):
    hw, hs = wplans
    A = inputs.gaussian(n, 300 + n)
    for p in POWERS:
        for log in (True, False):
            Mw, sw = run_gpu(hw, A, p, log_scale=log)
            Ms, ss = run_gpu(hs, A, p, log_scale=log)
            assert np.array_equal(Mw, Ms) and sw == ss, (n, p, log)
    for p in (2, 17, 1000):
        M, s = run_gpu(hw, A, p)
        err, tol, _ = check_against_oracle(M, s, A, p, seed=n)
        assert err <= tol, (n, p, err, tol)


@pytest.mark.parametrize("n", [5, 40, 64, 100, 128])
def test_power_wg_non_finite_inputs_match_tiles(wplans, n):
    # NaN and +-inf inputs: the running matrix's padding is kept zero, so
    # the values (NaNs in the same places) and the log2 scale are the
    # tiles'.
    hw, hs = wplans
    for j, bad in enumerate((np.nan, np.inf, -np.inf)):
        A = inputs.gaussian(n, 940 + 3 * n + j)
        A[(3 * j) % n, (7 + j) % n] = bad
        for p in (2, 3, 17):
            Mw, sw = run_gpu(hw, A, p)
            Ms, ss = run_gpu(hs, A, p)
            assert np.array_equal(Mw, Ms, equal_nan=True) and sw == ss, (n, p, j)


def test_power_wg_scaled_inputs_and_alias(wplans):
    hw, hs = wplans
    for k in (70, -70, 120):
        A = np.ldexp(inputs.gaussian(100, 5), k).astype(np.float32)
        Mw, sw = run_gpu(hw, A, 37)
        Ms, ss = run_gpu(hs, A, 37)
        assert np.array_equal(Mw, Ms) and sw == ss, k
    A = inputs.gaussian(77, 9)
    Mw, sw = run_gpu(hw, A, 55, out_is_input=True)
    Ms, ss = run_gpu(hs, A, 55)
    assert np.array_equal(Mw, Ms) and sw == ss


def test_power_wg_exact_structure(wplans):
    hw, _ = wplans
    # permutations: P^p = P_{sigma^p} exactly
    for n in (7, 64, 128):
        sigma = inputs.permutation_perm(n, n)
        tau, base, e = np.arange(n), sigma.copy(), 999
        while e:
            if e & 1:
                tau = base[tau]
            base = base[base]
            e >>= 1
        M, s = run_gpu(hw, inputs.permutation_matrix(sigma), 999)
        assert np.array_equal(oracle.to_value(M, s), inputs.permutation_matrix(tau).astype(np.float64))
    # nilpotent shift vanishes at its index, not before
    J = inputs.shift_matrix(40)
    M, s = run_gpu(hw, J, 40)
    assert s == 0 and not np.any(M)
    M, s = run_gpu(hw, J, 39)
    assert np.array_equal(oracle.to_value(M, s), np.eye(40, k=39))
    # all-ones 2^k: 1^p = N^(p-1) 1, log2 scale k p beyond float64's range
    M, s = run_gpu(hw, inputs.ones_matrix(128), 1000)
    assert s == 7 * 1000 and np.all(M == 2.0 ** -7)
    # zero matrix and NaN
    M, s = run_gpu(hw, np.zeros((50, 50), np.float32), 9)
    assert s == 0 and not np.any(M)
    A = inputs.gaussian(20, 1)
    A[3, 4] = np.nan
    M, _ = run_gpu(hw, A, 5, log_scale=False)
    assert np.isnan(M).any()


def test_power_wg_falls_back_above_its_size(wplans):
    # forced on a plan, sizes beyond 128 take the per-size product kernels
    hw, _ = wplans
    A = inputs.gaussian(200, 3)
    M, s = run_gpu(hw, A, 17)
    err, tol, _ = check_against_oracle(M, s, A, 17)
    assert err <= tol
