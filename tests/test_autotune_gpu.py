"""GPU tests of the single-matrix product picks of mpow_plan_autotune: for
every 256-wide size bucket the tuner times the product kernels of the plan's
mode that add each output's products in the per-size default's order, so a
tuned plan must give the untuned plan's bits; the choices are cached per GPU
model and mode."""
import numpy as np
import pytest

from paper_1204_3052_amd import inputs, mpow

from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

F32_CANDIDATES = {mpow.MPOW_KERNEL_GEMM_F32_256x128_DMA, mpow.MPOW_KERNEL_GEMM_F32_256,
                  mpow.MPOW_KERNEL_GEMM_F32_128_DMA, mpow.MPOW_KERNEL_GEMM_F32_64_DMA}


def test_fp32_picks_tuned_cached_and_bit_identical(tmp_path):
    import torch
    assert torch.cuda.is_available()
    cache = str(tmp_path / "picks.txt")
    ht = mpow.mpow_plan_create(0, 2048, 0, mpow.MPOW_FP32, 0)
    hd = mpow.mpow_plan_create(0, 2048, 0, mpow.MPOW_FP32, 0)
    h2 = mpow.mpow_plan_create(0, 2048, 0, mpow.MPOW_FP32, 0)
    try:
        small = {n: mpow.mpow_plan_kernel_for(ht, n) for n in (1, 64, 100, 512, 767)}
        print("  [gpu] mpow_plan_autotune (float32 picks up to n = 2048)", flush=True)
        mpow.mpow_plan_autotune(ht, cache, mpow.MPOW_TUNE_FORCE)
        for n, k in small.items():  # below n = 768 nothing is tuned
            assert mpow.mpow_plan_kernel_for(ht, n) == k, n
        assert mpow.mpow_plan_kernel_for(ht, 64) == mpow.MPOW_KERNEL_POWER_WG
        picks = {n: mpow.mpow_plan_kernel_for(ht, n) for n in range(768, 2049, 256)}
        assert set(picks.values()) <= F32_CANDIDATES, picks
        lines = open(cache).read().splitlines()
        assert lines[0].startswith("mpow-tune ") and lines[0].endswith("mode=0")
        assert sorted(int(l.split()[1]) for l in lines[1:]) == list(range(768, 2049, 256))
        # the cached choices load into another plan
        mpow.mpow_plan_autotune(h2, cache, 0)
        assert {n: mpow.mpow_plan_kernel_for(h2, n) for n in picks} == picks
        # same accumulation order: the tuned plan gives the default plan's bits
        for n, p in ((768, 17), (1000, 5), (1536, 3), (2048, 2)):
            A = inputs.gaussian(n, 800 + n)
            Mt, st = run_gpu(ht, A, p)
            Md, sd = run_gpu(hd, A, p)
            assert np.array_equal(Mt, Md) and st == sd, n
    finally:
        for h in (ht, hd, h2):
            mpow.mpow_plan_destroy(h)


@pytest.mark.parametrize("mode", [mpow.MPOW_BF16X3, mpow.MPOW_FP16X3])
def test_split_picks_tuned_and_bit_identical(tmp_path, mode):
    import torch
    assert torch.cuda.is_available()
    cache = str(tmp_path / "split.txt")
    ht = mpow.mpow_plan_create(0, 1024, 0, mode, 0)
    hd = mpow.mpow_plan_create(0, 1024, 0, mode, 0)
    try:
        print(f"  [gpu] mpow_plan_autotune (mode {mode} picks up to n = 1024)", flush=True)
        mpow.mpow_plan_autotune(ht, cache, mpow.MPOW_TUNE_FORCE)
        allowed = {mpow.MPOW_BF16X3: {mpow.MPOW_KERNEL_GEMM_BF16X3_128, mpow.MPOW_KERNEL_GEMM_BF16X3_256},
                   mpow.MPOW_FP16X3: {mpow.MPOW_KERNEL_GEMM_F16X3_128, mpow.MPOW_KERNEL_GEMM_F16X3_256}}[mode]
        picks = {n: mpow.mpow_plan_kernel_for(ht, n) for n in (1, 200, 256, 300, 700, 1024)}
        assert set(picks.values()) <= allowed, picks
        assert open(cache).read().splitlines()[0].endswith(f"mode={mode}")
        for n, p in ((200, 9), (700, 17), (1024, 3)):
            A = inputs.gaussian(n, 900 + n)
            Mt, st = run_gpu(ht, A, p)
            Md, sd = run_gpu(hd, A, p)
            assert np.array_equal(Mt, Md) and st == sd, n
        # a cache of another mode does not apply: the plan tunes afresh
        mpow.mpow_plan_autotune(hd, cache, 0)
        hf = mpow.mpow_plan_create(0, 1024, 0, mpow.MPOW_FP32, 0)
        try:
            mpow.mpow_plan_autotune(hf, cache, 0)
            assert open(cache).read().splitlines()[0].endswith("mode=0")
        finally:
            mpow.mpow_plan_destroy(hf)
    finally:
        mpow.mpow_plan_destroy(ht)
        mpow.mpow_plan_destroy(hd)
