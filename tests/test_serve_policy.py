"""CPU tests of the request server's admission and batching policy, run by
the library's own scheduler against a simulated executor
(mpow_srv_simulate): no device is touched."""
import numpy as np
import pytest

from paper_1204_3052_amd import inputs, mpow

FP32, BF16X3 = mpow.MPOW_FP32, mpow.MPOW_BF16X3


@pytest.fixture(scope="module", autouse=True)
def lib():
    import os
    if not os.path.exists(mpow.LIB_PATH):
        from paper_1204_3052_amd import build
        build.build(verbose=False)
    mpow._load()


def ws(n, mode):
    return mpow.mpow_workspace_bytes(n, 0, mode)


def trace(rate, duration, seed, n_hi=2048, p_hi=1 << 20):
    t, ns, ps, split = inputs.poisson_trace(rate, duration, seed, n_hi=n_hi, p_hi=p_hi)
    return [(float(a), int(n), int(p), BF16X3 if s else FP32) for a, n, p, s in zip(t, ns, ps, split)]


def test_budget_never_exceeded_and_all_complete():
    reqs = trace(2000, 1.0, 0)
    budget = 6 * ws(2048, BF16X3)
    res, peak = mpow.mpow_srv_simulate(reqs, budget, n_streams=4, plain_flops=4e13, batch_flops=4e13)
    assert peak <= budget
    assert all(r["status"] == mpow.MPOW_SUCCESS for r in res)
    assert all(r["t_end"] >= r["t_start"] >= r["t_admit"] >= a[0] for r, a in zip(res, reqs))


def test_large_requests_admitted_in_arrival_order():
    reqs = trace(2000, 0.5, 1)
    res, _ = mpow.mpow_srv_simulate(reqs, 3 * ws(2048, BF16X3), n_streams=2, plain_flops=2e13)
    admits = [r["t_admit"] for r in res if r["route"] == 0]
    assert len(admits) > 100
    assert all(b >= a for a, b in zip(admits, admits[1:]))


def test_small_requests_batched_while_others_run():
    # small FP32 requests arriving while batches run leave together in the
    # next batch (continuous batching); batches run one after another, and
    # at most two are in flight at once
    reqs = [(i * 1e-5, 64 + 16 * (i % 4), 100, FP32) for i in range(200)]
    res, peak = mpow.mpow_srv_simulate(reqs, 1 << 30, batch_flops=1e11)
    assert peak == 0 and all(r["route"] == 1 for r in res)
    groups = {}
    for r in res:
        groups.setdefault((r["t_admit"], r["t_start"], r["t_end"]), []).append(r)
    keys = sorted(groups, key=lambda k: k[1])
    assert 3 <= len(keys) < 50  # far fewer launches than requests
    assert max(len(v) for v in groups.values()) > 10
    for a, b in zip(keys, keys[1:]):
        assert b[1] >= a[2] - 1e-12  # one batch after another
    for k in keys:
        in_flight = sum(1 for o in keys if o[0] <= k[0] < o[2])
        assert in_flight <= 2


def test_batch_capacity_respected():
    reqs = [(0.0, 32, 17, FP32)] * 100
    res, _ = mpow.mpow_srv_simulate(reqs, 1 << 30, batch_cap=16, batch_flops=1e12)
    groups = {}
    for r in res:
        groups.setdefault(r["t_start"], 0)
        groups[r["t_start"]] += 1
    assert max(groups.values()) == 16 and sum(groups.values()) == 100


def test_request_larger_than_budget_rejected():
    reqs = [(0.0, 2048, 17, FP32), (0.1, 256, 3, BF16X3), (0.2, 64, 5, FP32)]
    res, _ = mpow.mpow_srv_simulate(reqs, ws(1024, FP32))
    assert res[0]["status"] == mpow.MPOW_ERR_BUDGET
    assert res[1]["status"] == mpow.MPOW_SUCCESS and res[2]["status"] == mpow.MPOW_SUCCESS


def test_head_of_line_waits_for_memory_small_ones_flow():
    big = ws(2048, FP32)
    budget = big + ws(512, FP32)  # room for one large request at a time
    reqs = [(0.0, 2048, 1 << 20, FP32), (0.001, 2048, 1 << 20, FP32)]
    reqs += [(0.002 + 1e-4 * i, 32, 9, FP32) for i in range(50)]
    res, peak = mpow.mpow_srv_simulate(reqs, budget, n_streams=4, plain_flops=1e13, batch_flops=1e13)
    assert peak <= budget
    assert res[1]["t_admit"] >= res[0]["t_end"] - 1e-12  # second waits for the first's memory
    assert max(r["t_end"] for r in res[2:]) < res[0]["t_end"]  # small requests did not wait


def test_no_starvation_under_sustained_load():
    reqs = trace(1500, 2.0, 2, n_hi=1024)
    res, _ = mpow.mpow_srv_simulate(reqs, 4 * ws(1024, BF16X3), n_streams=4, plain_flops=1e14,
                                    batch_flops=5e13)
    wait = np.array([r["t_admit"] - a[0] for r, a in zip(res, reqs)])
    assert np.all(np.isfinite(wait)) and wait.max() < 0.5


def test_simulate_rejects_bad_input():
    with pytest.raises(mpow.MpowError):
        mpow.mpow_srv_simulate([(1.0, 32, 2, FP32), (0.5, 32, 2, FP32)], 1 << 20)  # unsorted
    with pytest.raises(mpow.MpowError):
        mpow.mpow_srv_simulate([(0.0, 0, 2, FP32)], 1 << 20)
    with pytest.raises(mpow.MpowError):
        mpow.mpow_srv_simulate([(0.0, 8, -1, FP32)], 1 << 20)


def test_server_create_without_gpu_fails_cleanly():
    import ctypes
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    lib = mpow._load()
    assert lib.mpow_srv_create(ctypes.byref(h), 0, 64, 1 << 20, 2, 16, 0) == mpow.MPOW_ERR_DEVICE
    assert lib.mpow_srv_create(ctypes.byref(h), 0, 0, 1 << 20, 2, 16, 0) == mpow.MPOW_ERR_INVALID
    assert lib.mpow_srv_destroy(None) == mpow.MPOW_SUCCESS
