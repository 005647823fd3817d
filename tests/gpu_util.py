"""Helpers for GPU tests: run the library through its C ABI on numpy inputs.

Tolerances are the stated bars of oracle/tolerance.py: a result passes when
its relative Frobenius error against the FP64 oracle is at most
max(ABS, FACTOR * floor), floor being the oracle's own sensitivity to
float32-sized input noise.
"""
from __future__ import annotations

import numpy as np

import oracle
from paper_1204_3052_amd import inputs, mpow

from oracle.tolerance import (  # noqa: F401  (the stated bars live beside the oracle)
    BF16X3_ABS_TOL, BF16X3_FLOOR_FACTOR, FP32_ABS_TOL, FP32_FLOOR_FACTOR, tol_fp32, tol_mode)


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
