"""FP64 CPU oracle for the matrix exponential e^A (test infrastructure only).

Only the tests, the smoke check and the benchmark's oracle leg may import
this module; the GPU library never does.

e^A is defined by its series, e^A = sum over k >= 0 of A^k / k!.  The oracle
writes that definition out with the squaring identity e^A = (e^(A/2^j))^(2^j):

* j = max(0, floor(log2 ||A||_F) + 2), so that B = A * 2^-j (exact) has
  ||B||_F < 1/2;
* T = sum of B^k / k! for k = 0, 1, ... in float64, each term the previous
  one times B divided by k, until a term's Frobenius norm falls below 2^-60
  of the sum's (the rest of the series is then below float64 resolution);
* e^A = T^(2^j) by the power oracle (j squarings with power-of-two
  normalisation), returned as (M, s) with e^A = M * 2^s, ||M||_F in [1, 2).

The input is float32 widened exactly to float64.
"""
from __future__ import annotations

import numpy as np

from .mpow_oracle import frobenius_exponent, mpow_binary


def expm_squarings(A: np.ndarray) -> int:
    """j = max(0, floor(log2 ||A||_F) + 2); 0 for a zero matrix."""
    e = frobenius_exponent(A)
    return 0 if e is None else max(0, e + 2)


def taylor(B: np.ndarray) -> np.ndarray:
    """sum_k B^k / k! in float64, until the terms no longer matter."""
    B = np.asarray(B, dtype=np.float64)
    n = B.shape[0]
    T = np.eye(n)
    term = np.eye(n)
    for k in range(1, 200):
        term = term @ B / k
        T = T + term
        if np.linalg.norm(term) <= 2.0 ** -60 * np.linalg.norm(T):
            break
    return T


def expm(A: np.ndarray):
    """(M, s) with e^A = M * 2^s."""
    A = np.asarray(A, dtype=np.float64)
    j = expm_squarings(A)  # 0 when the norm is zero or not finite
    T = taylor(np.ldexp(A, -j))
    return mpow_binary(T, 2 ** j)
