"""GPU tests of the request server: mixed requests (small batched FP32, large
FP32, BF16X3) submitted together overlap on the device; each result must be
bit-identical to the same request run alone, meet its oracle tolerance, and
the arena must never exceed the budget."""
import numpy as np
import pytest

import oracle
from paper_1204_3052_amd import inputs, mpow

from gpu_util import tol_mode

pytestmark = pytest.mark.gpu

FP32, BF16X3, FP16X3 = mpow.MPOW_FP32, mpow.MPOW_BF16X3, mpow.MPOW_FP16X3


def request_set():
    reqs = []
    rng = np.random.default_rng(11)
    for i in range(48):
        n = int(rng.choice([16, 48, 100, 176, 256]))
        reqs.append((n, int(rng.integers(2, 3000)), FP32))
    for n in (300, 512, 640, 1024, 1024):
        reqs.append((n, int(rng.integers(2, 1 << 20)), FP32))
    for n in (64, 200, 512, 768, 1024):
        reqs.append((n, int(rng.integers(2, 5000)), BF16X3))
    reqs.append((333, 77, FP16X3))
    order = rng.permutation(len(reqs))
    return [reqs[k] for k in order]


class Buffers:
    def __init__(self, reqs, seed):
        import torch
        self.A = [torch.from_numpy(inputs.gaussian(n, seed + i)).cuda() for i, (n, _, _) in enumerate(reqs)]
        self.out = [torch.full_like(a, float("nan")) for a in self.A]
        self.scale = torch.full((len(reqs),), -1.0, dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()


def submit(srv, buf, reqs, idx):
    n, p, mode = reqs[idx]
    return mpow.mpow_srv_submit(srv, buf.A[idx].data_ptr(), n, p, mode, buf.out[idx].data_ptr(),
                                buf.scale[idx:idx + 1].data_ptr())


@pytest.fixture(scope="module")
def server():
    import torch
    assert torch.cuda.is_available()
    mpow._load()
    budget = 3 * mpow.mpow_workspace_bytes(1024, 0, BF16X3)
    srv = mpow.mpow_srv_create(0, 1024, budget, n_streams=3, max_batch=64)
    yield srv, budget
    mpow.mpow_srv_destroy(srv)


def test_alone_equals_in_mix(server):
    srv, budget = server
    reqs = request_set()
    mix = Buffers(reqs, 700)
    print(f"  [gpu] server mix of {len(reqs)} requests", flush=True)
    ids = [submit(srv, mix, reqs, i) for i in range(len(reqs))]
    mpow.mpow_srv_wait_idle(srv, 120.0)
    comp = {c["id"]: c for c in mpow.mpow_srv_poll(srv)}
    assert set(ids) <= set(comp) and all(comp[i]["status"] == 0 for i in ids)
    # continuous batching: small FP32 requests shared launches
    starts = [comp[i]["t_start"] for i, r in zip(ids, reqs) if r[0] <= 256 and r[2] == FP32]
    assert len(set(starts)) < len(starts)
    # overlap: some requests ran concurrently
    spans = sorted((comp[i]["t_start"], comp[i]["t_end"]) for i in ids)
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    st = mpow.mpow_srv_stats(srv)
    assert st["arena_peak"] <= budget and st["queued"] == 0

    alone = Buffers(reqs, 700)
    for i in range(len(reqs)):
        submit(srv, alone, reqs, i)
        mpow.mpow_srv_wait_idle(srv, 60.0)
    mpow.mpow_srv_poll(srv)
    for i, (n, p, mode) in enumerate(reqs):
        a, b = mix.out[i].cpu().numpy(), alone.out[i].cpu().numpy()
        assert np.array_equal(a, b), (n, p, mode)
        assert mix.scale[i].item() == alone.scale[i].item()

    # tolerance against the oracle for a sample of requests
    for i, (n, p, mode) in enumerate(reqs):
        if n > 512 or i % 3:
            continue
        A = mix.A[i].cpu().numpy()
        ref = oracle.mpow_binary(A, p)
        err = oracle.rel_err(mix.out[i].cpu().numpy(), mix.scale[i].item(), *ref)
        floor = oracle.floor_estimate(A, p, inputs.relative_signs(n, i), ref=ref)
        assert err <= tol_mode(mode, floor), (n, p, mode, err)


def test_budget_rejection_and_stats(server):
    import torch
    srv, budget = server
    small = mpow.mpow_srv_create(0, 2048, mpow.mpow_workspace_bytes(512, 0, FP32), n_streams=1,
                                 max_batch=0)
    try:
        A = torch.zeros((1024, 1024), device="cuda")
        with pytest.raises(mpow.MpowError) as e:
            mpow.mpow_srv_submit(small, A.data_ptr(), 1024, 3, FP32, A.data_ptr())
        assert e.value.status == mpow.MPOW_ERR_BUDGET
        B = torch.from_numpy(inputs.gaussian(256, 1)).cuda()
        out = torch.empty_like(B)
        mpow.mpow_srv_submit(small, B.data_ptr(), 256, 17, FP32, out.data_ptr())
        mpow.mpow_srv_wait_idle(small, 30.0)
        st = mpow.mpow_srv_stats(small)
        assert st["rejected"] == 1 and st["completed"] == 1 and st["arena_in_use"] == 0
        with pytest.raises(mpow.MpowError) as e:
            mpow.mpow_srv_submit(small, B.data_ptr(), 4096, 3, FP32, out.data_ptr())  # n > max_n
        assert e.value.status == mpow.MPOW_ERR_INVALID
    finally:
        mpow.mpow_srv_destroy(small)
