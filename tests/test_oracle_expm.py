"""Pins of the matrix-exponential oracle (CPU): an independent library
routine (scipy's Pade-based expm), closed forms (diagonal, nilpotent shift,
rotation generators, 1 x 1), and the group identity e^A e^-A = I."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1204_3052_amd import inputs


def value(Ms):
    M, s = Ms
    return np.ldexp(M, s)


@pytest.mark.parametrize("n,scale", [(1, 1.0), (7, 0.01), (50, 0.3), (100, 1.0), (100, 8.0), (64, 40.0)])
def test_against_scipy_expm(n, scale):
    A = (inputs.gaussian(n, 10 + n) * scale).astype(np.float32)
    R = scipy.linalg.expm(A.astype(np.float64))
    V = value(oracle.expm(A))
    assert np.linalg.norm(V - R) <= 1e-12 * np.linalg.norm(R)


def test_diagonal_closed_form():
    d = np.linspace(-20.0, 20.0, 41).astype(np.float32)
    V = value(oracle.expm(np.diag(d)))
    assert np.allclose(np.diag(V), np.exp(d.astype(np.float64)), rtol=1e-13, atol=0)
    assert not np.any(V - np.diag(np.diag(V)))


@pytest.mark.parametrize("t", [0.5, 3.0, 11.0])
def test_nilpotent_shift_closed_form(t):
    n = 12
    J = inputs.shift_matrix(n).astype(np.float64) * t
    V = value(oracle.expm(J.astype(np.float32)))
    E = np.zeros((n, n))
    for k in range(n):
        E += np.eye(n, k=k) * (t ** k / math.factorial(k))
    assert np.allclose(V, E, rtol=1e-13, atol=0)


def test_rotation_generators_closed_form():
    ts = [0.25, 1.0, 2.5, 7.0]
    n = 2 * len(ts)
    A = np.zeros((n, n), np.float32)
    for b, t in enumerate(ts):
        A[2 * b, 2 * b + 1] = -t
        A[2 * b + 1, 2 * b] = t
    V = value(oracle.expm(A))
    for b, t in enumerate(ts):
        t = float(np.float32(t))
        blk = V[2 * b:2 * b + 2, 2 * b:2 * b + 2]
        expect = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
        assert np.allclose(blk, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("x", [-30.0, -1.5, 0.0, 1e-3, 2.0, 60.0])
def test_scalar(x):
    V = value(oracle.expm(np.array([[x]], np.float32)))
    # a few float64 roundings per squaring (at most 7 squarings here)
    assert abs(V[0, 0] - math.exp(float(np.float32(x)))) <= 2e-14 * math.exp(float(np.float32(x)))


def test_zero_is_identity():
    assert np.array_equal(value(oracle.expm(np.zeros((9, 9), np.float32))), np.eye(9))


@pytest.mark.parametrize("scale", [0.5, 3.0])
def test_inverse_identity(scale):
    A = (inputs.gaussian(60, 3) * scale).astype(np.float32)
    P = value(oracle.expm(A)) @ value(oracle.expm(-A))
    assert np.linalg.norm(P - np.eye(60)) <= 1e-11 * 60


def test_squarings_keep_B_below_one_half():
    for scale in (1e-3, 0.7, 5.0, 300.0):
        A = (inputs.gaussian(40, 1) * scale).astype(np.float32)
        j = oracle.expm_squarings(A)
        assert np.linalg.norm(np.ldexp(A.astype(np.float64), -j)) < 0.5
        assert j == 0 or np.linalg.norm(np.ldexp(A.astype(np.float64), -(j - 2))) >= 0.5
