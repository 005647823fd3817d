"""Helpers for GPU tests: run the library through its C ABI on numpy inputs.

Tolerance (float32 products): a result passes when its relative Frobenius
error against the FP64 oracle is at most max(1e-5, 64 * floor), where floor is
the oracle's own relative change when every input entry moves by a random
relative +-2^-24 (the problem's sensitivity to float32-sized input noise).
At large p the power is ill-conditioned and no float32 method can reach 1e-5;
the floor term then takes over.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_1204_3052_amd import inputs, mpow

FP32_ABS_TOL = 1e-5
FP32_FLOOR_FACTOR = 64.0
# BF16 hi/lo halves carry about 16 bits of each operand: a looser stated bound.
BF16X3_ABS_TOL = 2e-4
BF16X3_FLOOR_FACTOR = 1024.0


def tol_fp32(floor: float) -> float:
    return max(FP32_ABS_TOL, FP32_FLOOR_FACTOR * floor)


def tol_mode(mode: int, floor: float) -> float:
    """Stated tolerance per product mode (FP16X3 shares the float32 bound)."""
    if mode == mpow.MPOW_BF16X3:
        return max(BF16X3_ABS_TOL, BF16X3_FLOOR_FACTOR * floor)
    return tol_fp32(floor)


def run_gpu(plan_handle: int, A_np: np.ndarray, p: int, log_scale: bool = True, out_is_input=False):
    """Returns (out, s) as numpy / float; s is None when log_scale is False."""
    import torch
    n = A_np.shape[0]
    A = torch.from_numpy(np.ascontiguousarray(A_np, dtype=np.float32)).cuda()
    out = A if out_is_input else torch.empty_like(A)
    s = torch.full((1,), -12345.0, dtype=torch.float64, device=A.device) if log_scale else None
    stream = torch.cuda.current_stream().cuda_stream
    print(f"  [gpu] mpow_run n={n} p={p} log={log_scale}", flush=True)
    mpow.mpow_run(plan_handle, A.data_ptr(), n, p, out.data_ptr(), s.data_ptr() if s is not None else None,
                  stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (float(s.item()) if s is not None else None)


def check_against_oracle(M, s, A_np, p, seed=0, ref=None):
    """Relative error of (M, s) vs the oracle and the tolerance it must meet."""
    if ref is None:
        ref = oracle.mpow_binary(A_np, p)
    M_ref, s_ref = ref
    err = oracle.rel_err(M, s, M_ref, s_ref)
    floor = oracle.floor_estimate(A_np, p, inputs.relative_signs(A_np.shape[0], 1000 + seed), ref=ref)
    return err, tol_fp32(floor), floor
