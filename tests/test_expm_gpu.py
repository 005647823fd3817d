"""GPU parity of the matrix exponential (mpow_expm) against the FP64 oracle,
through the C ABI: random matrices of several norms and ragged sizes within
the exponential's stated bar (oracle/tolerance.py: the float32 bar, or the
2^j growth of the j squarings), closed forms (zero, diagonal, rotation generators,
nilpotent shift), e^A e^-A = I, caller-chosen squarings, and the argument
checks."""
import math

import numpy as np
import pytest

import oracle
from oracle.tolerance import tol_expm
from paper_1204_3052_amd import inputs, mpow

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eplan():
    h = mpow.mpow_plan_create(0, 1100, 0, mpow.MPOW_FP32, mpow.MPOW_FLAG_EXPM)
    yield h
    mpow.mpow_plan_destroy(h)


def run_expm(h, A_np, squarings=-1, log_scale=True, out_is_input=False):
    import torch
    n = A_np.shape[0]
    A = torch.from_numpy(np.ascontiguousarray(A_np, dtype=np.float32)).cuda()
    out = A if out_is_input else torch.empty_like(A)
    s = torch.full((1,), -12345.0, dtype=torch.float64, device=A.device) if log_scale else None
    print(f"  [gpu] mpow_expm n={n} squarings={squarings}", flush=True)
    mpow.mpow_expm(h, A.data_ptr(), n, out.data_ptr(), s.data_ptr() if s is not None else None, squarings,
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), (float(s.item()) if s is not None else None)


def value(M, s):
    return np.ldexp(M.astype(np.float64), int(s))


def check(h, A, seed, squarings=-1):
    M, s = run_expm(h, A, squarings)
    ref = oracle.expm(A)
    err = oracle.rel_err(M, s, *ref)
    pert = oracle.perturbed(A, inputs.relative_signs(A.shape[0], 5000 + seed))
    Rp = oracle.expm(pert)
    floor = oracle.rel_err(Rp[0], Rp[1], *ref)
    j = oracle.expm_squarings(A) if squarings < 0 else squarings
    tol = tol_expm(floor, j)
    print(f"    n={A.shape[0]} norm={np.linalg.norm(A):.2e} err={err:.3e} tol={tol:.3e}")
    assert err <= tol, (A.shape[0], err, tol)
    return M, s


@pytest.mark.parametrize("n", [1, 2, 33, 100, 300, 513, 1030])
@pytest.mark.parametrize("scale", [0.05, 1.0, 8.0])
def test_expm_parity(eplan, n, scale):
    # ||A||_F ~ scale * sqrt(n): from far below 1/2 (no squarings) to ~260
    A = (inputs.gaussian(n, 70 + n) * scale).astype(np.float32)
    check(eplan, A, n)


@pytest.mark.parametrize("n", [300, 1028])
def test_expm_tile_shapes_bit_identical(eplan, n):
    # The Taylor products' identity-adding epilogue on the LDS-DMA tiles
    # (scales applied to the sums) and on the 128 x 128 tile (scales applied
    # on load) give the same bits; all meet the bar.
    A = (inputs.gaussian(n, 170 + n) * 4.0).astype(np.float32)
    runs = []
    for k in (mpow.MPOW_KERNEL_GEMM_F32_128, mpow.MPOW_KERNEL_GEMM_F32_256, mpow.MPOW_KERNEL_GEMM_F32_64_DMA,
              mpow.MPOW_KERNEL_GEMM_F32_128_DMA, mpow.MPOW_KERNEL_GEMM_F32_256x128_DMA):
        mpow.mpow_plan_set_kernel(eplan, k)
        try:
            runs.append(check(eplan, A, n))
        finally:
            mpow.mpow_plan_set_kernel(eplan, -1)
    M0, s0 = runs[0]
    for M1, s1 in runs[1:]:
        assert s0 == s1 and np.array_equal(M0, M1)


def test_expm_zero_is_identity(eplan):
    M, s = run_expm(eplan, np.zeros((9, 9), np.float32))
    assert np.array_equal(value(M, s), np.eye(9))
    out, _ = run_expm(eplan, np.zeros((5, 5), np.float32), log_scale=False)
    assert np.array_equal(out, np.eye(5, dtype=np.float32))


def test_expm_diagonal(eplan):
    d = np.linspace(-10.0, 10.0, 64).astype(np.float32)
    M, s = run_expm(eplan, np.diag(d))
    V = value(M, s)
    assert np.allclose(np.diag(V), np.exp(d.astype(np.float64)), rtol=2e-5, atol=0)
    assert np.max(np.abs(V - np.diag(np.diag(V)))) <= 1e-6 * np.max(np.abs(V))


def test_expm_rotation_generators(eplan):
    ts = [0.25, 1.0, 2.5, 7.0, 20.0]
    n = 2 * len(ts)
    A = np.zeros((n, n), np.float32)
    for b, t in enumerate(ts):
        A[2 * b, 2 * b + 1], A[2 * b + 1, 2 * b] = -t, t
    out, _ = run_expm(eplan, A, log_scale=False)
    for b, t in enumerate(ts):
        t = float(np.float32(t))
        blk = out[2 * b:2 * b + 2, 2 * b:2 * b + 2]
        expect = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
        assert np.allclose(blk, expect, rtol=0, atol=2e-5), (t, blk)


def test_expm_nilpotent_shift(eplan):
    n, t = 12, 3.0
    J = inputs.shift_matrix(n) * np.float32(t)
    out, _ = run_expm(eplan, J, log_scale=False)
    E = np.zeros((n, n))
    for k in range(n):
        E += np.eye(n, k=k) * (t ** k / math.factorial(k))
    assert np.allclose(out, E, rtol=1e-5, atol=1e-7)


def test_expm_inverse_identity(eplan):
    A = (inputs.gaussian(200, 3) * 2.0).astype(np.float32)
    Mp, sp = run_expm(eplan, A)
    Mm, sm = run_expm(eplan, -A)
    P = value(Mp, sp) @ value(Mm, sm)
    assert np.linalg.norm(P - np.eye(200)) <= 1e-4 * math.sqrt(200)


def test_expm_caller_squarings(eplan):
    # more squarings than needed stays accurate; j = 0 on a small matrix too
    A = (inputs.gaussian(128, 9) * 0.2).astype(np.float32)  # ||A||_F ~ 2.3
    for j in (4, 7, 10):
        check(eplan, A, j, squarings=j)
    B = (inputs.gaussian(64, 9) * 0.01).astype(np.float32)
    check(eplan, B, 1, squarings=0)


def test_expm_output_aliases_input(eplan):
    A = (inputs.gaussian(100, 4)).astype(np.float32)
    M0, s0 = run_expm(eplan, A)
    M1, s1 = run_expm(eplan, A, out_is_input=True)
    assert s0 == s1 and np.array_equal(M0, M1)


def test_expm_deterministic(eplan):
    A = (inputs.gaussian(300, 5) * 3.0).astype(np.float32)
    M0, s0 = run_expm(eplan, A)
    M1, s1 = run_expm(eplan, A)
    assert s0 == s1 and np.array_equal(M0, M1)


def test_expm_argument_checks(eplan):
    import torch
    A = torch.zeros((16, 16), device="cuda")
    for j in (-2, 63):
        with pytest.raises(mpow.MpowError) as e:
            mpow.mpow_expm(eplan, A.data_ptr(), 16, A.data_ptr(), None, j, None)
        assert e.value.status == mpow.MPOW_ERR_INVALID
    for mode, flags in ((mpow.MPOW_FP32, 0), (mpow.MPOW_FP16X3, mpow.MPOW_FLAG_EXPM)):
        h = mpow.mpow_plan_create(0, 16, 0, mode, flags)
        try:
            with pytest.raises(mpow.MpowError) as e:
                mpow.mpow_expm(h, A.data_ptr(), 16, A.data_ptr(), None, -1, None)
            assert e.value.status == mpow.MPOW_ERR_UNSUPPORTED
        finally:
            mpow.mpow_plan_destroy(h)
