"""FP64 CPU oracle for A^p (test infrastructure only).

Only tests, the smoke check and the benchmark's oracle legs (which time the
oracle for the CPU baseline and check GPU results against it) may import
this package.  The GPU library never does, and the two share no code.
"""
from .expm_oracle import expm, expm_squarings, taylor  # noqa: F401
from .mpow_oracle import (  # noqa: F401
    exact_int_power,
    floor_estimate,
    floor_estimate_rows,
    frobenius_exponent,
    gemm_count,
    matmul,
    matmul_naive,
    mpow_binary,
    mpow_naive,
    mpow_rows,
    naive_threads,
    normalize,
    perturbed,
    rel_err,
    set_naive_threads,
    row_rel_errs,
    schedule,
    to_value,
)
