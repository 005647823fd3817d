"""Seeded synthetic inputs for matrix-power runs.

This module only draws numbers.  It holds none of the power method's
arithmetic, so both the FP64 oracle and the GPU path can take their inputs
from it.  Every generator uses NumPy's PCG64 (`numpy.random.default_rng`)
with an explicit seed; matrices are drawn in float64 and handed out as
contiguous row-major float32 arrays, which is the element type the library
computes with.

The paper times dense square matrices of sizes 64..512 raised to powers
64..1024 (section 5.2, its timing tables) but never states what values the
matrices hold.  The distributions below stand in for those unstated inputs:

* ``row_stochastic`` - uniform [0,1) entries, each row divided by its sum;
  every power stays row-stochastic, so the row sums are a checkable invariant.
* ``gaussian`` - i.i.d. N(0,1)/sqrt(N) entries; spectral radius near 1, so
  powers neither explode nor vanish quickly.
* structured matrices with closed-form powers (permutation, nilpotent shift,
  all-ones, diagonal, Fibonacci and rotation blocks) used as exact checks.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(seed))


def row_stochastic(n: int, seed: int) -> np.ndarray:
    """U[0,1) entries, each row scaled (in float64) to sum to 1, then float32."""
    u = _rng(seed).random((n, n), dtype=np.float64)
    u /= u.sum(axis=1, keepdims=True)
    return np.ascontiguousarray(u.astype(np.float32))


def gaussian(n: int, seed: int) -> np.ndarray:
    """i.i.d. N(0,1)/sqrt(n) entries as float32."""
    g = _rng(seed).standard_normal((n, n), dtype=np.float64)
    g *= 1.0 / math.sqrt(n)
    return np.ascontiguousarray(g.astype(np.float32))


def small_integers(n: int, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Integer entries uniform in [lo, hi], as float32 (exact)."""
    a = _rng(seed).integers(lo, hi + 1, size=(n, n))
    return np.ascontiguousarray(a.astype(np.float32))


def permutation_perm(n: int, seed: int) -> np.ndarray:
    """A random permutation sigma of range(n) (int64)."""
    return _rng(seed).permutation(n).astype(np.int64)


def permutation_matrix(sigma: np.ndarray) -> np.ndarray:
    """P with P[i, sigma[i]] = 1 (row i has its one in column sigma[i])."""
    n = len(sigma)
    P = np.zeros((n, n), dtype=np.float32)
    P[np.arange(n), sigma] = 1.0
    return P


def shift_matrix(n: int) -> np.ndarray:
    """Nilpotent shift J: ones on the first superdiagonal."""
    J = np.zeros((n, n), dtype=np.float32)
    if n > 1:
        J[np.arange(n - 1), np.arange(1, n)] = 1.0
    return J


def ones_matrix(n: int) -> np.ndarray:
    return np.ones((n, n), dtype=np.float32)


def diagonal_matrix(d: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.diag(np.asarray(d, dtype=np.float32)))


def fibonacci_blocks(n: int) -> np.ndarray:
    """[[1,1],[1,0]] repeated along the diagonal; a trailing 1x1 block is [1]."""
    A = np.zeros((n, n), dtype=np.float32)
    for b in range(0, n - 1, 2):
        A[b, b] = A[b, b + 1] = A[b + 1, b] = 1.0
    if n % 2 == 1:
        A[n - 1, n - 1] = 1.0
    return A


def rotation_blocks(n: int, theta: float) -> np.ndarray:
    """2x2 rotations R(theta) along the diagonal (float32 of the float64 values)."""
    A = np.zeros((n, n), dtype=np.float64)
    c, s = math.cos(theta), math.sin(theta)
    for b in range(0, n - 1, 2):
        A[b, b], A[b, b + 1], A[b + 1, b], A[b + 1, b + 1] = c, -s, s, c
    if n % 2 == 1:
        A[n - 1, n - 1] = 1.0
    return np.ascontiguousarray(A.astype(np.float32))


def relative_signs(n: int, seed: int) -> np.ndarray:
    """Random +-1 per entry (float64), used to perturb an input by +-2^-24 relative."""
    return np.where(_rng(seed).random((n, n)) < 0.5, -1.0, 1.0)


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int, size, step: int = 1) -> np.ndarray:
    """round(exp(U(ln lo, ln hi))) to a multiple of `step`, clamped to [lo, hi]."""
    x = np.exp(rng.uniform(math.log(lo), math.log(hi), size=size))
    v = np.rint(x / step).astype(np.int64) * step
    return np.clip(v, lo, hi)


def ragged_batch(count: int, seed: int, n_lo: int = 16, n_hi: int = 256,
                 n_step: int = 16, p_lo: int = 2, p_hi: int = 1000):
    """Sizes and exponents of a ragged batch: N uniform over multiples of
    `n_step` in [n_lo, n_hi], p log-uniform in [p_lo, p_hi]."""
    rng = _rng(seed)
    ns = rng.integers(n_lo // n_step, n_hi // n_step + 1, size=count) * n_step
    ps = log_uniform_int(rng, p_lo, p_hi, count)
    return ns.astype(np.int64), ps.astype(np.int64)


def poisson_trace(rate: float, duration: float, seed: int, n_lo: int = 32,
                  n_hi: int = 2048, n_step: int = 16, p_lo: int = 2,
                  p_hi: int = 1 << 20, split_fraction: float = 0.5):
    """Open-loop request trace: exponential inter-arrival times at `rate`/s
    for `duration` s; N log-uniform on multiples of `n_step`; p log-uniform;
    a fraction `split_fraction` of requests asks for the split-precision mode.
    Returns (arrival_s, n, p, split_flag) arrays."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * duration * 1.5) + 16)
    t = np.cumsum(gaps)
    t = t[t < duration]
    m = len(t)
    ns = log_uniform_int(rng, n_lo, n_hi, m, step=n_step)
    ps = log_uniform_int(rng, p_lo, p_hi, m)
    split = rng.random(m) < split_fraction
    return t, ns, ps, split
