"""GPU tests of the torch helpers of the Python binding (mpow.run with a
mode, mpow.run_batched, mpow.Server).  They only marshal arguments, so each
must give the bits of the raw C entry point it forwards to."""
import numpy as np
import pytest

from paper_1204_3052_amd import inputs, mpow

pytestmark = pytest.mark.gpu

MODES = [mpow.MPOW_FP32, mpow.MPOW_FP16X3, mpow.MPOW_BF16X3, mpow.MPOW_BF16X6]


def _raw_run(mode, A, p):
    import torch
    n = A.shape[0]
    h = mpow.mpow_plan_create(0, n, 0, mode, 0)
    try:
        out = torch.empty_like(A)
        s = torch.empty(1, dtype=torch.float64, device=A.device)
        mpow.mpow_run(h, A.data_ptr(), n, p, out.data_ptr(), s.data_ptr(),
                      torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        mpow.mpow_plan_destroy(h)
    return out.cpu().numpy(), float(s.item())


@pytest.mark.parametrize("mode", MODES)
def test_run_with_mode_matches_c_path(mode):
    import torch
    n, p = 300, 37
    A = torch.from_numpy(inputs.gaussian(n, 900 + mode)).cuda()
    print(f"  [gpu] mpow.run mode={mode} n={n} p={p}", flush=True)
    M, s = mpow.run(A, p, mode=mode, return_scale=True)
    torch.cuda.synchronize()
    M_raw, s_raw = _raw_run(mode, A, p)
    assert np.array_equal(M.cpu().numpy(), M_raw) and float(s.item()) == s_raw
    with mpow.Plan(n, mode=mode) as plan:
        M2, s2 = mpow.run(A, p, plan=plan, return_scale=True)
        torch.cuda.synchronize()
        assert np.array_equal(M2.cpu().numpy(), M_raw) and float(s2.item()) == s_raw
        other = mpow.MPOW_FP32 if mode != mpow.MPOW_FP32 else mpow.MPOW_BF16X3
        with pytest.raises(ValueError):
            mpow.run(A, p, plan=plan, mode=other)


def test_run_batched_matches_c_path():
    import torch
    ns, ps = inputs.ragged_batch(40, 5)
    As = [torch.from_numpy(inputs.gaussian(int(n), 2000 + i)).cuda() for i, n in enumerate(ns)]
    print(f"  [gpu] mpow.run_batched count={len(As)}", flush=True)
    outs, s = mpow.run_batched(As, ps, return_scale=True)
    torch.cuda.synchronize()
    h = mpow.mpow_plan_create(0, 256, len(As), mpow.MPOW_FP32, 0)
    try:
        ref = [torch.empty_like(A) for A in As]
        sr = torch.empty(len(As), dtype=torch.float64, device="cuda")
        mpow.mpow_run_batched(h, len(As), [A.data_ptr() for A in As], [int(n) for n in ns],
                              [int(p) for p in ps], [o.data_ptr() for o in ref], sr.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
    finally:
        mpow.mpow_plan_destroy(h)
    for i in range(len(As)):
        assert np.array_equal(outs[i].cpu().numpy(), ref[i].cpu().numpy()), i
    assert np.array_equal(s.cpu().numpy(), sr.cpu().numpy())
    # unscaled outputs, caller-provided, through a caller's plan
    with mpow.Plan(256, max_batch=len(As)) as plan:
        mine = [torch.full_like(A, float("nan")) for A in As]
        got = mpow.run_batched(As, ps, plan=plan, outs=mine)
        torch.cuda.synchronize()
        assert got is mine
    sv = sr.cpu().numpy()
    for i in range(len(As)):
        # the unscaled output is M * 2^s rounded once to float32
        want = np.ldexp(ref[i].cpu().numpy().astype(np.float64), int(sv[i])).astype(np.float32)
        assert np.array_equal(mine[i].cpu().numpy(), want), i
    assert mpow.run_batched([], []) == []


def test_server_class_matches_run():
    import torch
    reqs = [(64, 100, mpow.MPOW_FP32), (200, 1000, mpow.MPOW_FP32), (512, 33, mpow.MPOW_FP32),
            (320, 77, mpow.MPOW_BF16X3), (96, 5, mpow.MPOW_BF16X3)]
    As = [torch.from_numpy(inputs.gaussian(n, 3000 + i)).cuda() for i, (n, _, _) in enumerate(reqs)]
    budget = 2 * mpow.mpow_workspace_bytes(512, 0, mpow.MPOW_BF16X3)
    print(f"  [gpu] mpow.Server with {len(reqs)} requests", flush=True)
    with mpow.Server(512, budget, n_streams=2, max_batch=16) as srv:
        handles = [srv.submit(A, p, mode=mode, return_scale=True) for A, (n, p, mode) in zip(As, reqs)]
        srv.wait_idle(60.0)
        done = srv.poll()
        assert sorted(c["id"] for c in done) == sorted(h[0] for h in handles)
        assert all(c["status"] == mpow.MPOW_SUCCESS for c in done)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["arena_peak"] <= budget
    route = {c["id"]: c["route"] for c in done}
    for (rid, out, s), A, (n, p, mode) in zip(handles, As, reqs):
        # small float32 requests leave through the batched kernel, the rest
        # through mpow_run's kernels on a stream of their own
        if route[rid] == 1:
            ref, sr = mpow.run_batched([A], [p], return_scale=True)
            torch.cuda.synchronize()
            M_raw, s_raw = ref[0].cpu().numpy(), float(sr[0].item())
        else:
            M_raw, s_raw = _raw_run(mode, A, p)
        assert np.array_equal(out.cpu().numpy(), M_raw), (n, p, mode)
        assert float(s.item()) == s_raw
    assert sorted(route.values()) == [0, 0, 0, 1, 1]
