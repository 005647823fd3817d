"""FP64 CPU oracle for the integer matrix power A^p.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's oracle legs (timing the oracle for the CPU baseline, checking GPU
results against it) may import this module.  It shares no code,
headers, tables or helpers with the GPU library, and the GPU library never
imports it.

What it computes (the paper, section 4): the p-th power of a dense square
matrix, A^p = A.A...A (p factors), with A^0 = I.

* ``mpow_naive`` is the paper's naive method (section 4.1): start from A and
  multiply by A again p-1 times, each product being the plain three-loop
  product of section 4.1 (the C helper in ``naive_matmul.c``).
* ``mpow_binary`` is the paper's method (section 4.3): reach the power with a
  number of products logarithmic in p, by repeated squaring.  The bits of p
  are taken from the most significant one down: each later bit squares the
  running matrix, and a set bit then multiplies it by A once more
  (left-to-right binary exponentiation).  It uses floor(log2 p) squarings and
  popcount(p)-1 multiplications.  NumPy's float64 matmul serves as the
  product primitive.
* ``mpow_rows`` gives selected rows of A^p by repeated row-vector times
  matrix products, for sizes where the full power is too costly on a CPU.

Readings where the paper is silent (each is listed in the design notes):

* Element type.  The input is float32 (the library's type); the oracle widens
  it exactly to float64 and computes in float64, so input rounding is not
  counted as error.
* Range.  Powers of the paper's sizes overflow any floating type, so after
  every product the running matrix X is multiplied by 2^-e with
  e = floor(log2 ||X||_F), an exact power of two, and e is added to an integer
  log2 scale s.  Results are returned as (M, s) with A^p = M * 2^s and
  ||M||_F in [1, 2).  Scaling by a power of two is exact, so where nothing
  overflows or underflows the scaled and unscaled computations agree bit for
  bit.
* Zero.  A zero matrix, or a power that vanishes (nilpotent A), gives M = 0
  and s = 0; no scaling is applied to a zero matrix.  A non-finite norm
  (NaN/Inf entries) disables scaling and the values propagate.
* p = 0 gives (I, 0); p = 1 gives A scaled; p < 0 is rejected.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _naive_lib():
    global _lib
    if _lib is None:
        from . import build as _build
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        lib.oracle_naive_matmul_f64.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p, ctypes.c_int64]
        lib.oracle_naive_matmul_f64.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        _lib = lib
    return _lib


# --------------------------------------------------------------------------
# products
# --------------------------------------------------------------------------

def matmul_naive(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """The section 4.1 three-loop product in float64 (C helper)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    n = X.shape[0]
    assert X.shape == (n, n) and Y.shape == (n, n)
    C = np.empty((n, n), dtype=np.float64)
    if n:
        _naive_lib().oracle_naive_matmul_f64(X.ctypes.data, Y.ctypes.data, C.ctypes.data, n)
    return C


def matmul(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """float64 product by NumPy's matmul (a library primitive)."""
    return np.matmul(np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64))


def naive_threads() -> int:
    return int(_naive_lib().oracle_num_threads())


def set_naive_threads(n: int) -> None:
    """Thread count of the three-loop product (1: the paper's sequential CPU method)."""
    _naive_lib().oracle_set_threads(int(n))


# --------------------------------------------------------------------------
# power-of-two normalisation
# --------------------------------------------------------------------------

def frobenius_exponent(X: np.ndarray):
    """e = floor(log2 ||X||_F), or None when ||X||_F is zero or not finite.

    With S = sum of squares = m * 2^q (m in [0.5, 1)), floor(log2 S) = q - 1
    and floor(log2 sqrt(S)) = floor((q - 1) / 2), which is exact given S.
    """
    S = float(np.sum(np.square(np.asarray(X, dtype=np.float64))))
    if S == 0.0 or not math.isfinite(S):
        return None
    _, q = math.frexp(S)
    return (q - 1) // 2


def frobenius_exponent_rows(X: np.ndarray) -> list:
    return [frobenius_exponent(X[i]) for i in range(X.shape[0])]


def normalize(X: np.ndarray, s: int):
    """Return (X * 2^-e, s + e) for e = floor(log2 ||X||_F); unchanged if zero."""
    e = frobenius_exponent(X)
    if e is None:
        return X, s
    return np.ldexp(X, -e), s + e


def _finish(X: np.ndarray, s: int):
    if not np.any(X) and np.all(np.isfinite(X)):
        return np.zeros_like(X), 0
    return X, s


# --------------------------------------------------------------------------
# the power
# --------------------------------------------------------------------------

def schedule(p: int) -> list:
    """Products of left-to-right binary exponentiation for p >= 2:
    for every bit of p below the most significant one, 'S' (square) and,
    when that bit is set, 'M' (multiply by A).  Empty for p in {0, 1}."""
    if p < 0:
        raise ValueError("negative power")
    ops = []
    if p < 2:
        return ops
    for bit in range(p.bit_length() - 2, -1, -1):
        ops.append("S")
        if (p >> bit) & 1:
            ops.append("M")
    return ops


def gemm_count(p: int) -> int:
    """Number of products ``mpow_binary`` performs: floor(log2 p) + popcount(p) - 1."""
    return len(schedule(p))


def _identity(n: int) -> np.ndarray:
    return np.eye(n, dtype=np.float64)


def mpow_naive(A: np.ndarray, p: int, product=matmul_naive):
    """Section 4.1: p-1 chained products X <- X.A starting from X = A.

    Returns (M, s) with A^p = M * 2^s."""
    if p < 0:
        raise ValueError("negative power")
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if p == 0:
        return _identity(n), 0
    An, sA = normalize(A, 0)
    X, s = An.copy(), sA
    for _ in range(p - 1):
        X = product(X, An)
        s = s + sA
        X, s = normalize(X, s)
    return _finish(X, s)


def mpow_binary(A: np.ndarray, p: int, product=matmul):
    """Section 4.3: left-to-right binary exponentiation.

    X starts as A (scaled).  For each bit of p below the leading one:
    X <- X.X (the true value's scale doubles: s <- 2s), then, if the bit is
    set, X <- X.A (s <- s + s_A).  After every product X is renormalised.
    Returns (M, s) with A^p = M * 2^s."""
    if p < 0:
        raise ValueError("negative power")
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if p == 0:
        return _identity(n), 0
    An, sA = normalize(A, 0)
    X, s = An.copy(), sA
    for op in schedule(p):
        if op == "S":
            X = product(X, X)
            s = 2 * s
        else:
            X = product(X, An)
            s = s + sA
        X, s = normalize(X, s)
    return _finish(X, s)


def mpow_rows(A: np.ndarray, p: int, rows) -> tuple:
    """Rows `rows` of A^p by p-1 row-vector times matrix products.

    Row r of A^p is e_r^T A^p = (row r of A) . A ... A.  Each row carries its
    own power-of-two scale.  Returns (R, s) with row k of A^p equal to
    R[k] * 2^s[k]; a vanished row gives zeros and scale 0."""
    if p < 0:
        raise ValueError("negative power")
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    rows = list(rows)
    if p == 0:
        return _identity(n)[rows], [0] * len(rows)
    An, sA = normalize(A, 0)
    V = A[rows].copy()
    s = [0] * len(rows)

    def renorm(V, s):
        for k in range(V.shape[0]):
            e = frobenius_exponent(V[k])
            if e is not None:
                V[k] = np.ldexp(V[k], -e)
                s[k] += e
        return V, s

    V, s = renorm(V, s)
    for _ in range(p - 1):
        V = matmul(V, An)
        s = [x + sA for x in s]
        V, s = renorm(V, s)
    for k in range(V.shape[0]):
        if not np.any(V[k]) and np.all(np.isfinite(V[k])):
            s[k] = 0
    return V, s


# --------------------------------------------------------------------------
# comparison helpers
# --------------------------------------------------------------------------

def to_value(M: np.ndarray, s: int) -> np.ndarray:
    """M * 2^s in float64 (overflows to +-inf / underflows to 0 as float64 does)."""
    return np.ldexp(np.asarray(M, dtype=np.float64), int(s))


def rel_err(M: np.ndarray, s, M_ref: np.ndarray, s_ref) -> float:
    """||M * 2^(s - s_ref) - M_ref||_F / ||M_ref||_F, in float64.

    When M_ref is zero the result is 0 if M is exactly zero, else inf."""
    M = np.asarray(M, dtype=np.float64)
    M_ref = np.asarray(M_ref, dtype=np.float64)
    den = float(np.linalg.norm(M_ref))
    if den == 0.0:
        return 0.0 if not np.any(M) else math.inf
    d = float(s) - float(s_ref)
    if abs(d) > 2000:
        return math.inf
    diff = np.ldexp(M, int(d)) - M_ref
    return float(np.linalg.norm(diff)) / den


def row_rel_errs(R: np.ndarray, s_rows, R_ref: np.ndarray, s_ref_rows) -> list:
    return [rel_err(R[k], s_rows[k], R_ref[k], s_ref_rows[k]) for k in range(R.shape[0])]


def perturbed(A: np.ndarray, signs: np.ndarray) -> np.ndarray:
    """A with every entry moved by a relative +-2^-24 (float64, not rounded)."""
    A = np.asarray(A, dtype=np.float64)
    return A * (1.0 + signs * 2.0 ** -24)


def floor_estimate(A: np.ndarray, p: int, signs: np.ndarray, ref=None) -> float:
    """Sensitivity of A^p to float32-sized input noise: the oracle's relative
    change when each entry of A moves by a random relative +-2^-24.
    `ref` may pass the already computed (M, s) of A^p."""
    M, s = mpow_binary(A, p) if ref is None else ref
    Mp, sp = mpow_binary(perturbed(A, signs), p)
    return rel_err(Mp, sp, M, s)


def floor_estimate_rows(A: np.ndarray, p: int, rows, signs: np.ndarray, ref=None) -> list:
    """Per-row floor_estimate of rows `rows` of A^p (the row method);
    `ref` may pass the already computed (R, s) of those rows."""
    R, s = mpow_rows(A, p, rows) if ref is None else ref
    Rp, sp = mpow_rows(perturbed(A, signs), p, rows)
    return row_rel_errs(Rp, sp, R, s)


def exact_int_power(A_int, p: int):
    """Exact A^p of an integer matrix with Python integers (p-1 products)."""
    n = len(A_int)
    A = [[int(v) for v in row] for row in A_int]
    if p == 0:
        return [[1 if i == j else 0 for j in range(n)] for i in range(n)]
    X = [row[:] for row in A]
    for _ in range(p - 1):
        X = [[sum(X[i][k] * A[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    return X
