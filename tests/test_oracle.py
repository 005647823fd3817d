"""Pins for the FP64 oracle (CPU only).

The paper prints timings but no values of any power, so the oracle is tied
to mathematics instead: closed forms, exact integer brute force, invariants,
special cases that reduce to library routines, and the exactness of
power-of-two scaling.  Each test names the mistake it would catch.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mpow_oracle as O
from paper_1204_3052_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "int_powers.txt")


def value(M, s):
    return O.to_value(M, s)


def abs_matrix_power_max(A_int, p):
    absA = [[abs(int(v)) for v in row] for row in A_int]
    P = O.exact_int_power(absA, p)
    return max(max(row) for row in P) if P else 0


# ---------------------------------------------------------------- schedule

@pytest.mark.parametrize("p", list(range(0, 300)) + [1000, 1023, 1024, 2 ** 20, 2 ** 20 - 1, 2 ** 40 + 7])
def test_schedule_reaches_p(p):
    # Replaying the schedule on the exponent alone must land on p, using
    # floor(log2 p) squarings and popcount(p)-1 multiplications.
    ops = O.schedule(p)
    e = 1 if p >= 1 else 0
    for op in ops:
        e = 2 * e if op == "S" else e + 1
    assert e == p
    if p >= 1:
        assert ops.count("S") == p.bit_length() - 1
        assert ops.count("M") == bin(p).count("1") - 1
        if ops:
            assert ops[0] == "S" and "MM" not in "".join(ops)


def test_gemm_counts_for_named_sizes():
    # G(p) = floor(log2 p) + popcount(p) - 1 for the exponents the benchmark uses.
    expect = {2: 1, 17: 5, 64: 6, 256: 8, 1000: 14, 1023: 18, 2 ** 20: 20, 2 ** 20 - 1: 38}
    for p, g in expect.items():
        assert O.gemm_count(p) == g


def test_paper_powers_take_log2_products():
    # Section 4.3: the method's product count is logarithmic in the power
    # rather than linear; the powers timed in section 5.2 are 64..1024, all
    # powers of two.
    for p in (64, 128, 256, 512, 1024):
        assert O.gemm_count(p) == int(math.log2(p))


# ---------------------------------------------------------- normalisation

def test_frobenius_exponent_exact_powers_of_two():
    for j in range(-40, 41, 7):
        X = np.zeros((3, 3))
        X[1, 2] = 2.0 ** j
        assert O.frobenius_exponent(X) == j
        X[0, 0] = 2.0 ** j  # norm 2^j * sqrt(2): still exponent j
        assert O.frobenius_exponent(X) == j
        X[2, 1] = X[2, 2] = 2.0 ** j  # norm 2^(j+1)
        assert O.frobenius_exponent(X) == j + 1


def test_frobenius_exponent_against_log2():
    rng = np.random.default_rng(5)
    for _ in range(200):
        X = rng.standard_normal((4, 5)) * 2.0 ** rng.integers(-300, 300)
        nrm = float(np.linalg.norm(X))
        lg = math.log2(nrm)
        if abs(lg - round(lg)) < 1e-9:
            continue
        assert O.frobenius_exponent(X) == math.floor(lg)


def test_frobenius_exponent_zero_and_nan():
    assert O.frobenius_exponent(np.zeros((4, 4))) is None
    X = np.ones((2, 2))
    X[0, 0] = np.nan
    assert O.frobenius_exponent(X) is None


# ---------------------------------------------------------- products

def test_naive_product_matches_definition_tiny():
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 7):
        X = rng.integers(-9, 10, (n, n)).astype(np.float64)
        Y = rng.integers(-9, 10, (n, n)).astype(np.float64)
        C = O.matmul_naive(X, Y)
        for i in range(n):
            for j in range(n):
                assert C[i, j] == sum(X[i, k] * Y[k, j] for k in range(n))


def test_naive_product_vs_numpy():
    X = inputs.gaussian(96, 3).astype(np.float64)
    Y = inputs.gaussian(96, 4).astype(np.float64)
    np.testing.assert_allclose(O.matmul_naive(X, Y), X @ Y, rtol=0, atol=1e-13)
    # order of operands matters: a transposed operand would be caught here
    assert not np.allclose(O.matmul_naive(X, Y), O.matmul_naive(Y, X))


# ---------------------------------------------------------- p = 0, 1

@pytest.mark.parametrize("fn", [O.mpow_binary, O.mpow_naive])
def test_power_zero_is_identity(fn):
    A = inputs.gaussian(9, 0)
    M, s = fn(A, 0)
    assert s == 0 and np.array_equal(M, np.eye(9))
    # also for a singular (zero) matrix
    M, s = fn(np.zeros((4, 4), np.float32), 0)
    assert s == 0 and np.array_equal(M, np.eye(4))


@pytest.mark.parametrize("fn", [O.mpow_binary, O.mpow_naive])
def test_power_one_is_input(fn):
    A = inputs.gaussian(17, 1) * np.float32(1e30)
    M, s = fn(A, 1)
    assert np.array_equal(value(M, s), A.astype(np.float64))
    assert 1.0 <= np.linalg.norm(M) < 2.0


def test_negative_power_rejected():
    with pytest.raises(ValueError):
        O.mpow_binary(np.eye(2), -1)
    with pytest.raises(ValueError):
        O.mpow_naive(np.eye(2), -3)


# ---------------------------------------------------------- exact brute force

def test_small_integer_brute_force():
    checked = 0
    for seed in range(12):
        n = [1, 2, 3, 4, 5, 8][seed % 6]
        A = inputs.small_integers(n, seed, -2, 2)
        Ai = A.astype(np.int64).tolist()
        for p in list(range(0, 13)) + [16, 31, 32, 33, 40]:
            if abs_matrix_power_max(Ai, p) >= 2 ** 53:
                continue
            exact = np.array(O.exact_int_power(Ai, p), dtype=object)
            for fn in (O.mpow_binary, O.mpow_naive):
                M, s = fn(A, p)
                got = value(M, s)
                assert np.array_equal(got, exact.astype(np.float64)), (seed, n, p, fn.__name__)
                checked += 1
    assert checked > 150


def test_golden_integer_powers():
    cases = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "case":
                n = int(tok[2])
                cases.append([tok[1], n, None, []])
            elif tok[0] == "A":
                cases[-1][2] = np.array([int(v) for v in tok[1:]], dtype=np.float32).reshape(n, n)
            elif tok[0] == "p":
                cases[-1][3].append((int(tok[1]), np.array([int(v) for v in tok[2:]], dtype=np.float64).reshape(n, n)))
    assert len(cases) == 3
    for name, n, A, rows in cases:
        for p, P in rows:
            for fn in (O.mpow_binary, O.mpow_naive):
                M, s = fn(A, p)
                assert np.array_equal(value(M, s), P), (name, p, fn.__name__)


# ---------------------------------------------------------- closed forms

@pytest.mark.parametrize("n,seed", [(5, 0), (16, 1), (64, 2), (97, 3)])
def test_permutation_powers_exact(n, seed):
    sigma = inputs.permutation_perm(n, seed)
    P = inputs.permutation_matrix(sigma)
    # order of sigma = lcm of cycle lengths
    seen = [False] * n
    order = 1
    for i in range(n):
        if not seen[i]:
            L, j = 0, i
            while not seen[j]:
                seen[j] = True
                j = sigma[j]
                L += 1
            order = order * L // math.gcd(order, L)
    for p in [0, 1, 2, 3, 7, 64, 100, order]:
        # (P^p)[i, tau[i]] = 1 with tau = sigma applied p times
        tau = np.arange(n)
        for _ in range(p):
            tau = sigma[tau]
        expect = inputs.permutation_matrix(tau).astype(np.float64)
        M, s = O.mpow_binary(P, p)
        assert np.array_equal(value(M, s), expect), p
    M, s = O.mpow_binary(P, order)
    assert np.array_equal(value(M, s), np.eye(n))


@pytest.mark.parametrize("n", [1, 2, 7, 32, 33])
def test_nilpotent_shift(n):
    J = inputs.shift_matrix(n)
    for k in range(0, n + 3):
        M, s = O.mpow_binary(J, k)
        if k >= n:
            assert s == 0 and not np.any(M), k
        else:
            assert np.array_equal(value(M, s), np.eye(n, k=k)), k
    # naive path vanishes too
    M, s = O.mpow_naive(J, n)
    assert s == 0 and not np.any(M)


def test_strictly_upper_triangular_vanishes_at_n():
    rng = np.random.default_rng(4)
    n = 12
    A = np.triu(rng.standard_normal((n, n)), k=1).astype(np.float32)
    M, s = O.mpow_binary(A, n - 1)
    assert np.any(M)
    M, s = O.mpow_binary(A, n)
    assert s == 0 and not np.any(M)


@pytest.mark.parametrize("k,p", [(0, 5), (1, 9), (4, 33), (7, 1000), (7, 64), (9, 1023)])
def test_all_ones(k, p):
    # 1^p = N^(p-1) 1 with N = 2^k, so M = 1/N and s = k*p, beyond float64
    # range for the larger cases.
    n = 2 ** k
    M, s = O.mpow_binary(inputs.ones_matrix(n), p)
    assert s == k * p
    assert np.array_equal(M, np.full((n, n), 2.0 ** -k))


def test_diagonal_powers_of_two_exact():
    d = np.array([2.0, -0.5, 4.0, -1.0, 0.25, 1.0], dtype=np.float32)
    D = inputs.diagonal_matrix(d)
    for p in (0, 1, 2, 5, 17, 63):
        M, s = O.mpow_binary(D, p)
        assert np.array_equal(value(M, s), np.diag(d.astype(np.float64) ** p)), p


def test_diagonal_general():
    d = np.array([1.1, -0.9, 0.7, 1.05, -1.2], dtype=np.float32)
    D = inputs.diagonal_matrix(d)
    for p in (3, 17, 256):
        M, s = O.mpow_binary(D, p)
        ref = np.diag(d.astype(np.float64) ** p)
        np.testing.assert_allclose(value(M, s), ref, rtol=p * 2e-16 * 4, atol=0)


def test_fibonacci_blocks_exact():
    F = [0, 1]
    while len(F) < 90:
        F.append(F[-1] + F[-2])
    A = inputs.fibonacci_blocks(7)
    for p in [1, 2, 3, 10, 35, 50, 77]:
        M, s = O.mpow_binary(A, p)
        V = value(M, s)
        for b in range(0, 6, 2):
            assert V[b, b] == F[p + 1] and V[b, b + 1] == F[p] and V[b + 1, b] == F[p] and V[b + 1, b + 1] == F[p - 1], p
        assert V[6, 6] == 1.0


def test_rotation_blocks():
    theta = 0.3
    A = inputs.rotation_blocks(6, theta).astype(np.float64)
    c, s_ = A[0, 0], A[1, 0]  # the float32-rounded rotation
    th = math.atan2(s_, c)
    r = math.hypot(c, s_)
    for p in (2, 17, 256, 1023):
        M, s = O.mpow_binary(A, p)
        V = value(M, s)
        rp = r ** p
        ref = np.array([[math.cos(p * th), -math.sin(p * th)], [math.sin(p * th), math.cos(p * th)]]) * rp
        np.testing.assert_allclose(V[0:2, 0:2], ref, atol=p * 1e-14 * rp)


def test_row_stochastic_row_sums():
    A = inputs.row_stochastic(64, 0)
    A64 = A.astype(np.float64)
    r0 = A64.sum(axis=1)  # float32 rounding moves the row sums off 1 slightly
    for p in (2, 17, 64, 256):
        M, s = O.mpow_binary(A, p)
        rs = value(M, s) @ np.ones(64)
        # A^p 1 = A^(p-1) (A 1): compare against the input's own row sums
        ref = np.linalg.matrix_power(A64, p - 1) @ r0
        np.testing.assert_allclose(rs, ref, rtol=1e-12)
        assert np.max(np.abs(rs - 1.0)) < 1e-5


# ---------------------------------------------------------- invariants

def test_semigroup_property():
    A = inputs.gaussian(48, 7)
    for m, n in [(1, 1), (3, 5), (17, 16), (100, 28)]:
        Mm, sm = O.mpow_binary(A, m)
        Mn, sn = O.mpow_binary(A, n)
        Mmn, smn = O.mpow_binary(A, m + n)
        prod = Mm @ Mn
        assert O.rel_err(prod, sm + sn, Mmn, smn) < 1e-12 * (m + n)


def test_naive_equals_binary_gaussian():
    A = inputs.gaussian(40, 11)
    for p in (2, 3, 17, 64, 100):
        Mb, sb = O.mpow_binary(A, p)
        Mn, sn = O.mpow_naive(A, p)
        assert O.rel_err(Mn, sn, Mb, sb) < 1e-13 * p


def test_symmetric_against_eigh():
    rng = np.random.default_rng(8)
    n = 50
    G = rng.standard_normal((n, n))
    S = ((G + G.T) / (2 * math.sqrt(n))).astype(np.float32)
    w, V = np.linalg.eigh(S.astype(np.float64))
    for p in (2, 17, 64, 255):
        ref = (V * w ** p) @ V.T
        M, s = O.mpow_binary(S, p)
        assert O.rel_err(value(M, s), 0, ref, 0) < 1e-11 * p


def test_against_numpy_matrix_power():
    A = inputs.gaussian(30, 2)
    for p in (0, 1, 2, 5, 17, 64):
        ref = np.linalg.matrix_power(A.astype(np.float64), p)
        M, s = O.mpow_binary(A, p)
        assert O.rel_err(value(M, s), 0, ref, 0) < 1e-13 * max(p, 1)


def test_scaled_equals_unscaled_bitwise():
    # Power-of-two scaling is exact: with the same product routine, the
    # scaled chains reproduce the unscaled ones bit for bit when nothing
    # overflows or underflows.
    A = inputs.gaussian(24, 9)
    A64 = A.astype(np.float64)
    for p in (2, 3, 6, 17, 45, 64):
        raw = A64.copy()
        for _ in range(p - 1):
            raw = O.matmul_naive(raw, A64)
        M, s = O.mpow_naive(A, p)
        assert np.array_equal(value(M, s), raw), p
        raw = A64.copy()
        for op in O.schedule(p):
            raw = O.matmul_naive(raw, raw if op == "S" else A64)
        M, s = O.mpow_binary(A, p, product=O.matmul_naive)
        assert np.array_equal(value(M, s), raw), p


@pytest.mark.parametrize("fn", [O.mpow_binary, O.mpow_naive])
def test_result_is_normalised(fn):
    A = inputs.gaussian(20, 3) * np.float32(37.0)
    for p in (1, 2, 9, 33):
        M, s = fn(A, p)
        assert 1.0 <= np.linalg.norm(M) < 2.0


def test_rows_match_full_power():
    A = inputs.gaussian(64, 13)
    rows = [0, 5, 63, 31]
    for p in (0, 1, 2, 17, 100):
        M, s = O.mpow_binary(A, p)
        R, sr = O.mpow_rows(A, p, rows)
        full = value(M, s)
        for k, r in enumerate(rows):
            assert O.rel_err(R[k], sr[k], full[r], 0) < 1e-13 * max(p, 1)


def test_rows_vanish_for_nilpotent():
    J = inputs.shift_matrix(10)
    R, s = O.mpow_rows(J, 10, [0, 3, 9])
    assert not np.any(R) and s == [0, 0, 0]
    R, s = O.mpow_rows(J, 4, [0, 5, 6])
    assert np.array_equal(O.to_value(R[0], s[0]), np.eye(10)[4])
    assert np.array_equal(O.to_value(R[1], s[1]), np.eye(10)[9])
    assert not np.any(R[2]) and s[2] == 0


# ---------------------------------------------------------- error metric, floor

def test_rel_err_metric():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((5, 5))
    assert O.rel_err(M, 3, M, 3) == 0.0
    assert O.rel_err(M * 2, 2, M, 3) == 0.0  # scale-invariant representation
    assert abs(O.rel_err(M * (1 + 1e-6), 0, M, 0) - 1e-6) < 1e-12
    assert O.rel_err(np.zeros((2, 2)), 5, np.zeros((2, 2)), 0) == 0.0
    assert O.rel_err(np.eye(2), 0, np.zeros((2, 2)), 0) == math.inf


def test_floor_estimate_grows_with_p():
    A = inputs.gaussian(64, 21)
    sg = inputs.relative_signs(64, 22)
    f2 = O.floor_estimate(A, 2, sg)
    f64 = O.floor_estimate(A, 64, sg)
    assert 1e-9 < f2 < 1e-6
    assert f64 > f2
    assert O.floor_estimate(inputs.ones_matrix(8), 17, inputs.relative_signs(8, 1)) < 1e-6


# ------------------------------------------- floor machinery: closed forms
#
# The floor term of every stated bar is the oracle's relative change under a
# relative +-u input perturbation, u = 2^-24 the unit roundoff of float32
# (half its machine epsilon).  These pins fix u, the perturbation, the power
# and the error metric against values computed independently of the oracle:
# exact rational arithmetic on diagonal matrices, and the first-order
# perturbation series of A^p on dense ones.  A perturbation of 2^-23 or
# 2^-22 (an epsilon in place of the unit roundoff) doubles or quadruples the
# floor and fails each of them.

from fractions import Fraction

U32 = float(np.finfo(np.float32).eps) / 2.0  # float32 unit roundoff, 2^-24


def _closed_form_diag_floor(signs, p):
    """sqrt(mean_i ((1 + s_i u)^p - 1)^2) in exact rational arithmetic."""
    u = Fraction(1, 2 ** 24)
    terms = [((1 + int(s) * u) ** p - 1) ** 2 for s in np.ravel(signs)]
    return math.sqrt(float(sum(terms) / len(terms)))


def test_perturbation_is_float32_unit_roundoff():
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((9, 9)) * 2.0 ** rng.integers(-40, 40, (9, 9))).astype(np.float32)
    sg = inputs.relative_signs(9, 4)
    P = O.perturbed(A, sg)
    A64 = A.astype(np.float64)
    rel = (P - A64) / A64
    assert U32 == 2.0 ** -24
    assert np.array_equal(rel, sg * U32)  # exact: entries are float32, u a power of two
    assert np.array_equal(O.perturbed(np.zeros((3, 3)), inputs.relative_signs(3, 1)), np.zeros((3, 3)))


@pytest.mark.parametrize("p", [1, 2, 3, 17, 64, 256, 1023])
def test_floor_estimate_scalar_identity_closed_form(p):
    # D = c I_n with signs s: the perturbed power is c^p diag((1 + s_i u)^p),
    # so the floor is the root mean square of (1 + s_i u)^p - 1, about p u.
    n = 6
    for c in (0.75, -1.5, 3.0):
        D = (np.eye(n) * c).astype(np.float32)
        sg = inputs.relative_signs(n, 10 + p)
        got = O.floor_estimate(D, p, sg)
        want = _closed_form_diag_floor(np.diag(sg), p)
        assert abs(got - want) <= 1e-7 * want, (c, p, got, want)
        # the same value with an epsilon of 2^-23 would be about twice as large
        assert abs(got - 2 * want) > 0.4 * want


@pytest.mark.parametrize("p", [1, 2, 5, 100, 1023])
def test_floor_estimate_one_by_one(p):
    for s in (-1.0, 1.0):
        got = O.floor_estimate(np.array([[0.625]], dtype=np.float32), p, np.array([[s]]))
        want = abs(float((1 + Fraction(int(s), 2 ** 24)) ** p - 1))
        assert abs(got - want) <= 1e-7 * want, (p, s, got, want)


@pytest.mark.parametrize("p", [2, 17, 256])
def test_floor_estimate_rows_diagonal_closed_form(p):
    # Row i of diag(d)^p only sees the perturbation of d_i: its relative
    # change is |(1 + s_ii u)^p - 1|.
    n = 8
    d = np.array([0.5, -0.5, 0.5, 0.5, -0.5, 0.5, -0.5, 0.5], dtype=np.float32)
    D = np.diag(d)
    sg = inputs.relative_signs(n, 40 + p)
    rows = [0, 3, 4, 7]
    got = O.floor_estimate_rows(D, p, rows, sg)
    for r, g in zip(rows, got):
        want = abs(float((1 + Fraction(int(sg[r, r]), 2 ** 24)) ** p - 1))
        assert abs(g - want) <= 1e-7 * want, (r, g, want)


def test_row_rel_errs_closed_form():
    # rows scaled by known factors (1 + delta_k) and carried with different
    # power-of-two scales: the row errors are |delta_k| exactly up to rounding
    rng = np.random.default_rng(8)
    R_ref = rng.standard_normal((4, 16))
    deltas = [3e-7, -1e-5, 0.0, 2.5e-3]
    shifts = [0, 3, -7, 60]
    R = np.stack([np.ldexp(R_ref[k] * (1 + deltas[k]), -shifts[k]) for k in range(4)])
    errs = O.row_rel_errs(R, shifts, R_ref, [0] * 4)
    for e, d in zip(errs, deltas):
        assert abs(e - abs(d)) <= 1e-12 + 1e-9 * abs(d), (e, d)


@pytest.mark.parametrize("p", [2, 17, 64])
def test_floor_estimate_rows_match_full_power(p):
    # The row method (p - 1 vector-matrix products) against the rows of the
    # binary method's full power: two different computations of the same
    # perturbed and unperturbed rows.
    n = 24
    A = inputs.gaussian(n, 50 + p)
    sg = inputs.relative_signs(n, 60 + p)
    rows = [0, 5, 11, 23]
    got = O.floor_estimate_rows(A, p, rows, sg)
    M, s = O.mpow_binary(A, p)
    Mp, sp = O.mpow_binary(O.perturbed(A, sg), p)
    V, Vp = O.to_value(M, s), O.to_value(Mp, sp)
    for r, g in zip(rows, got):
        want = float(np.linalg.norm(Vp[r] - V[r]) / np.linalg.norm(V[r]))
        assert abs(g - want) <= 1e-5 * want, (r, g, want)


@pytest.mark.parametrize("p", [2, 3, 17, 64])
def test_floor_estimate_first_order_series(p):
    # To first order in u, A^p moves by L = sum_{k=0}^{p-1} A^k E A^(p-1-k)
    # with E = u (A o S) (o: entrywise product): the floor is ||L|| / ||A^p||
    # up to terms of relative size about p u times the conditioning.  The
    # recurrence L_{m+1} = L_m A + A^m E gives L without the oracle's code.
    n = 12
    A = inputs.gaussian(n, 70 + p).astype(np.float64)
    sg = inputs.relative_signs(n, 80 + p)
    E = A * sg * U32
    P = np.eye(n)
    L = np.zeros((n, n))
    for _ in range(p):
        L = L @ A + P @ E
        P = P @ A
    want = float(np.linalg.norm(L) / np.linalg.norm(P))
    got = O.floor_estimate(A.astype(np.float32), p, sg)
    assert abs(got - want) <= 1e-3 * want, (p, got, want)


@pytest.mark.parametrize("eps", [2.0 ** -23, 2.0 ** -22, 2.0 ** -25])
def test_floor_pins_catch_a_wrong_perturbation(monkeypatch, eps):
    # Plant the slip in the oracle (an epsilon in place of the unit roundoff,
    # or half of it) and check that the closed forms above reject it.
    monkeypatch.setattr(O, "perturbed",
                        lambda A, signs: np.asarray(A, dtype=np.float64) * (1.0 + signs * eps))
    n, p = 6, 17
    D = (np.eye(n) * 0.75).astype(np.float32)
    sg = inputs.relative_signs(n, 10 + p)
    want = _closed_form_diag_floor(np.diag(sg), p)
    assert abs(O.floor_estimate(D, p, sg) - want) > 0.4 * want
    d = np.diag(np.full(8, 0.5, dtype=np.float32))
    sg8 = inputs.relative_signs(8, 42)
    got = O.floor_estimate_rows(d, p, [0], sg8)[0]
    want_row = abs(float((1 + Fraction(int(sg8[0, 0]), 2 ** 24)) ** p - 1))
    assert abs(got - want_row) > 0.4 * want_row
