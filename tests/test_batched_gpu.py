"""GPU tests of mpow_run_batched (ragged batch in one persistent launch).

Each matrix of a batch must equal its own mpow_run result bit for bit (both
paths accumulate every element in the same order), meet the oracle
tolerance, and stay the same when the graph is replayed with other work in
between."""
import numpy as np
import pytest

import oracle
from paper_1204_3052_amd import inputs, mpow

from gpu_util import run_gpu, tol_fp32

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plans():
    import torch
    assert torch.cuda.is_available()
    mpow._load()
    hb = mpow.mpow_plan_create(0, 256, 4096, mpow.MPOW_FP32, 0)
    hp = mpow.mpow_plan_create(0, 256, 0, mpow.MPOW_FP32, 0)
    # The batched kernel adds each output's products in the order of the
    # plain path's kernels without a K split: compare against one of those.
    mpow.mpow_plan_set_kernel(hp, mpow.MPOW_KERNEL_GEMM_F32_64)
    yield hb, hp
    mpow.mpow_plan_destroy(hb)
    mpow.mpow_plan_destroy(hp)


class Packed:
    """Matrices packed into one device buffer at 256-byte aligned offsets."""

    def __init__(self, mats):
        import torch
        self.ns = [m.shape[0] for m in mats]
        offs, o = [], 0
        for n in self.ns:
            offs.append(o)
            o += (n * n + 63) // 64 * 64
        host = np.zeros(o, np.float32)
        for m, off in zip(mats, offs):
            host[off:off + m.size] = m.ravel()
        self.dev = torch.from_numpy(host).cuda()
        self.out = torch.full_like(self.dev, np.nan)
        self.scale = torch.full((len(mats),), -777.0, dtype=torch.float64, device="cuda")
        self.offs = offs
        base, ob = self.dev.data_ptr(), self.out.data_ptr()
        self.a_ptrs = [base + 4 * off for off in offs]
        self.o_ptrs = [ob + 4 * off for off in offs]

    def result(self, i):
        n, off = self.ns[i], self.offs[i]
        return self.out[off:off + n * n].cpu().numpy().reshape(n, n), float(self.scale[i].item())


def run_batch(h, pk, ps, log_scale=True):
    import torch
    print(f"  [gpu] mpow_run_batched count={len(ps)}", flush=True)
    mpow.mpow_run_batched(h, len(ps), pk.a_ptrs, pk.ns, ps, pk.o_ptrs,
                          pk.scale.data_ptr() if log_scale else None,
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()


EDGE_N = [1, 2, 3, 5, 16, 17, 31, 32, 33, 63, 64, 65, 100, 128, 129, 200, 255, 256]
EDGE_P = [0, 1, 2, 3, 17, 100, 1000]


def edge_batch(seed):
    rng = np.random.default_rng(seed)
    mats, ps = [], []
    for i, n in enumerate(EDGE_N):
        for p in EDGE_P:
            mats.append(inputs.gaussian(n, 1000 * seed + 7 * i + p))
            ps.append(int(p))
    order = rng.permutation(len(mats))
    return [mats[k] for k in order], [ps[k] for k in order]


def test_batched_equals_plain_bitwise(plans):
    hb, hp = plans
    mats, ps = edge_batch(1)
    pk = Packed(mats)
    run_batch(hb, pk, ps)
    for i, (A, p) in enumerate(zip(mats, ps)):
        Mb, sb = pk.result(i)
        Mp, sp = run_gpu(hp, A, p)
        assert np.array_equal(Mb, Mp) and sb == sp, (A.shape[0], p)


# Every n a multiple of 4 (and the packed buffers 256-byte aligned): such a
# batch runs on the LDS-DMA instance, which must give the plain path's bits,
# also where an input's scale sends its first product down the operand-scaled
# path (entries scaled by 2^70 and 2^-70).
EDGE4_N = [4, 8, 12, 16, 20, 60, 64, 68, 100, 124, 128, 132, 192, 200, 252, 256]


def edge4_batch(seed):
    mats, ps = [], []
    for i, n in enumerate(EDGE4_N):
        for j, p in enumerate(EDGE_P):
            A = inputs.gaussian(n, 1000 * seed + 7 * i + p)
            if j % 3 == 1:
                A = np.ldexp(A, 70 if i % 2 else -70).astype(np.float32)
            mats.append(A)
            ps.append(int(p))
    order = np.random.default_rng(seed).permutation(len(mats))
    return [mats[k] for k in order], [ps[k] for k in order]


def test_batched_dma_instance_equals_plain_bitwise(plans):
    hb, hp = plans
    mats, ps = edge4_batch(4)
    pk = Packed(mats)
    run_batch(hb, pk, ps)
    for i, (A, p) in enumerate(zip(mats, ps)):
        Mb, sb = pk.result(i)
        Mp, sp = run_gpu(hp, A, p)
        assert np.array_equal(Mb, Mp) and sb == sp, (A.shape[0], p)


def test_batched_nonlog_equals_plain(plans):
    hb, hp = plans
    mats, ps = edge_batch(2)
    pk = Packed(mats)
    run_batch(hb, pk, ps, log_scale=False)
    for i, (A, p) in enumerate(zip(mats, ps)):
        ob, _ = pk.result(i)
        op, _ = run_gpu(hp, A, p, log_scale=False)
        assert np.array_equal(ob, op), (A.shape[0], p)


def test_batched_against_oracle(plans):
    hb, _ = plans
    mats, ps = edge_batch(3)
    pk = Packed(mats)
    run_batch(hb, pk, ps)
    for i, (A, p) in enumerate(zip(mats, ps)):
        M, s = pk.result(i)
        ref = oracle.mpow_binary(A, p)
        err = oracle.rel_err(M, s, *ref)
        floor = oracle.floor_estimate(A, p, inputs.relative_signs(A.shape[0], i), ref=ref)
        assert err <= tol_fp32(floor), (A.shape[0], p, err)


def test_batched_structured_exact(plans):
    hb, _ = plans
    mats, ps, expect = [], [], []
    for n in (16, 100, 256):
        sigma = inputs.permutation_perm(n, n)
        mats.append(inputs.permutation_matrix(sigma))
        ps.append(1000)
        tau, base, e = np.arange(n), sigma.copy(), 1000
        while e:
            if e & 1:
                tau = base[tau]
            base = base[base]
            e >>= 1
        expect.append(("perm", inputs.permutation_matrix(tau).astype(np.float64)))
        mats.append(inputs.shift_matrix(n))
        ps.append(n)
        expect.append(("zero", None))
    for k in (4, 7, 8):
        mats.append(inputs.ones_matrix(2 ** k))
        ps.append(33)
        expect.append(("ones", k))
    pk = Packed(mats)
    run_batch(hb, pk, ps)
    for i, (kind, ref) in enumerate(expect):
        M, s = pk.result(i)
        if kind == "perm":
            assert np.array_equal(oracle.to_value(M, s), ref)
        elif kind == "zero":
            assert s == 0 and not np.any(M)
        else:
            assert s == ref * 33 and np.all(M == 2.0 ** -ref)


def test_graph_replays_with_eager_work_between(plans):
    import torch
    hb, hp = plans
    mats, ps = edge_batch(4)
    pk = Packed(mats)
    run_batch(hb, pk, ps)
    first = [pk.result(i) for i in range(len(ps))]
    junk = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        pk.out.fill_(float("nan"))
        pk.scale.fill_(-1.0)
        junk = junk @ junk.T.contiguous() * 1e-3  # unrelated eager work on the stream
        torch.cuda.synchronize()
        run_batch(hb, pk, ps)
        for i in range(len(ps)):
            M, s = pk.result(i)
            assert np.array_equal(M, first[i][0]) and s == first[i][1], (rep, i)
    # new inputs of the same shapes through the same captured graph
    mats2 = [inputs.gaussian(m.shape[0], 99 + i) for i, m in enumerate(mats)]
    pk2 = Packed(mats2)
    run_batch(hb, pk2, ps)
    for i in range(0, len(ps), 7):
        M, s = pk2.result(i)
        Mp, sp = run_gpu(hp, mats2[i], ps[i])
        assert np.array_equal(M, Mp) and s == sp


def test_ragged_batch_4096(plans):
    # 4096 matrices, N uniform over multiples of 16 in [16, 256], p log-uniform
    # in [2, 1000], N(0,1)/sqrt(N) entries.
    hb, hp = plans
    ns, ps = inputs.ragged_batch(4096, 3)
    mats = [inputs.gaussian(int(n), 50000 + i) for i, n in enumerate(ns)]
    pk = Packed(mats)
    run_batch(hb, pk, [int(p) for p in ps])
    rng = np.random.default_rng(0)
    sample = rng.choice(4096, 24, replace=False)
    for i in sample:
        M, s = pk.result(i)
        Mp, sp = run_gpu(hp, mats[i], int(ps[i]))
        assert np.array_equal(M, Mp) and s == sp, (int(ns[i]), int(ps[i]))
    for i in sample[:8]:
        M, s = pk.result(i)
        ref = oracle.mpow_binary(mats[i], int(ps[i]))
        floor = oracle.floor_estimate(mats[i], int(ps[i]), inputs.relative_signs(int(ns[i]), int(i)), ref=ref)
        assert oracle.rel_err(M, s, *ref) <= tol_fp32(floor)
    allM = pk.out.cpu().numpy()
    assert np.isfinite(allM).all()


def test_batched_invalid_arguments(plans):
    import torch
    hb, hp = plans
    lib = mpow._load()
    A = torch.zeros(300 * 300, device="cuda")
    pk = Packed([np.zeros((4, 4), np.float32)])
    with pytest.raises(mpow.MpowError) as e:
        mpow.mpow_run_batched(hb, 1, [A.data_ptr()], [257], [2], [A.data_ptr()], None, None)
    assert e.value.status == mpow.MPOW_ERR_INVALID
    with pytest.raises(mpow.MpowError) as e:
        mpow.mpow_run_batched(hb, 1, pk.a_ptrs, pk.ns, [-1], pk.o_ptrs, None, None)
    assert e.value.status == mpow.MPOW_ERR_INVALID
    with pytest.raises(mpow.MpowError) as e:
        mpow.mpow_run_batched(hp, 1, pk.a_ptrs, pk.ns, [2], pk.o_ptrs, None, None)  # max_batch 0
    assert e.value.status == mpow.MPOW_ERR_INVALID
    mpow.mpow_run_batched(hb, 0, [], [], [], [], None, None)  # empty batch is fine
    torch.cuda.synchronize()


def test_default_table_is_panel_form(plans):
    # a plan starts with the streamed-panel whole-power form (shape 4) for
    # every size; tuning may replace it
    h = mpow.mpow_plan_create(0, 256, 8, mpow.MPOW_FP32, 0)
    try:
        assert mpow.mpow_plan_tile_table(h)[1:] == [4] * (mpow.TILE_TABLE_LEN - 1)
    finally:
        mpow.mpow_plan_destroy(h)


def test_tile_shapes_bit_identical(plans):
    hb, _ = plans
    mats, ps = edge_batch(5)
    pk = Packed(mats)
    saved = mpow.mpow_plan_tile_table(hb)
    results = []
    # all 128x128, all 64x64 (the instance without the large tile), a mix of
    # both in one launch, all 256x256 (the 8-wave instance), a mix of those,
    # the whole power per workgroup (resident, then streamed panels), and
    # mixes of every shape (several launch groups in one batch)
    L = mpow.TILE_TABLE_LEN
    tables = [[0] * L, [1] * L, [b % 2 for b in range(L)], [2] * L, [b % 3 for b in range(L)],
              [3] * L, [4] * L, [b % 5 for b in range(L)], [(b + 3) % 5 for b in range(L)]]
    for table in tables:
        mpow.mpow_plan_tile_table(hb, table)
        pk.out.fill_(float("nan"))
        run_batch(hb, pk, ps)
        results.append([pk.result(i) for i in range(len(ps))])
    mpow.mpow_plan_tile_table(hb, saved)
    for k in range(1, len(tables)):
        for i in range(len(ps)):
            assert np.array_equal(results[k][i][0], results[0][i][0]), (k, i)
            assert results[k][i][1] == results[0][i][1]


def test_autotune_and_cache(plans, tmp_path):
    hb, _ = plans
    cache = str(tmp_path / "tune.txt")
    print("  [gpu] mpow_plan_autotune", flush=True)
    mpow.mpow_plan_autotune(hb, cache, mpow.MPOW_TUNE_FORCE)
    table = mpow.mpow_plan_tile_table(hb)
    assert all(0 <= t < 5 for t in table)
    text = open(cache).read().splitlines()
    assert text[0].startswith("mpow-tune ") and len(text) == 17
    h2 = mpow.mpow_plan_create(0, 256, 16, mpow.MPOW_FP32, 0)
    try:
        mpow.mpow_plan_tile_table(h2, [1] * mpow.TILE_TABLE_LEN)
        mpow.mpow_plan_autotune(h2, cache, 0)  # loads the cached table
        assert mpow.mpow_plan_tile_table(h2)[1:] == table[1:]
    finally:
        mpow.mpow_plan_destroy(h2)
    for bad in (5, 7, -1):
        with pytest.raises(mpow.MpowError):
            mpow.mpow_plan_tile_table(hb, [bad] * mpow.TILE_TABLE_LEN)


@pytest.mark.parametrize("shape", [3, 4])
def test_whole_power_instance_equals_plain_bitwise(plans, shape):
    # the whole power per workgroup (tile shape 3: operands resident in LDS
    # up to n = 128; shape 4: streamed panels) on ragged sizes of any
    # alignment, and on multiple-of-4 sizes with 2^+-70-scaled inputs
    hb, hp = plans
    saved = mpow.mpow_plan_tile_table(hb)
    mpow.mpow_plan_tile_table(hb, [shape] * mpow.TILE_TABLE_LEN)
    try:
        for mats, ps in (edge_batch(6), edge4_batch(7)):
            pk = Packed(mats)
            run_batch(hb, pk, ps)
            for i, (A, p) in enumerate(zip(mats, ps)):
                Mb, sb = pk.result(i)
                Mp, sp = run_gpu(hp, A, p)
                assert np.array_equal(Mb, Mp) and sb == sp, (A.shape[0], p)
            pk.out.fill_(float("nan"))
            run_batch(hb, pk, ps, log_scale=False)
            for i, (A, p) in enumerate(zip(mats, ps)):
                if i % 5 == 0:
                    ob, _ = pk.result(i)
                    op, _ = run_gpu(hp, A, p, log_scale=False)
                    assert np.array_equal(ob, op), (A.shape[0], p)
    finally:
        mpow.mpow_plan_tile_table(hb, saved)


def test_panel_products_far_below_norm_one(plans):
    # Nearly nilpotent inputs A = J + 2^k G (J a single corner entry, so
    # J^2 = 0): the first product's norm is about 2^k times that of the
    # normalised input.  The streamed-panel form keeps a product in memory as
    # computed down to exponent -16 (k = -6) and stores it rescaled below
    # that (k = -20, -40); either way every result keeps the plain path's
    # bits and meets the oracle's bar.
    hb, hp = plans
    saved = mpow.mpow_plan_tile_table(hb)
    mpow.mpow_plan_tile_table(hb, [4] * mpow.TILE_TABLE_LEN)
    try:
        mats, ps = [], []
        for i, n in enumerate((16, 40, 64, 100, 128, 160, 200, 256)):
            for j, k in enumerate((-6, -20, -40)):
                A = np.ldexp(inputs.gaussian(n, 9100 + 10 * i + j).astype(np.float64), k)
                A[0, n - 1] += 1.0
                A = A.astype(np.float32)
                for p in (2, 3, 5, 17, 100):
                    mats.append(A)
                    ps.append(p)
        pk = Packed(mats)
        run_batch(hb, pk, ps)
        for i, (A, p) in enumerate(zip(mats, ps)):
            Mb, sb = pk.result(i)
            Mp, sp = run_gpu(hp, A, p)
            assert np.array_equal(Mb, Mp) and sb == sp, (A.shape[0], p, i)
            if i % 4 == 0:
                ref = oracle.mpow_binary(A, p)
                err = oracle.rel_err(Mb, sb, *ref)
                floor = oracle.floor_estimate(A, p, inputs.relative_signs(A.shape[0], i), ref=ref)
                assert err <= tol_fp32(floor), (A.shape[0], p, err)
    finally:
        mpow.mpow_plan_tile_table(hb, saved)


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_non_finite_inputs_match_plain(plans, shape):
    # A NaN or an infinity in the input spreads through the products; every
    # tile shape (the whole-power forms keep zero padding in their running
    # matrix, and the panel form sums it unmasked) gives the plain path's
    # values, NaNs in the same places, and the same log2 scale.
    hb, hp = plans
    saved = mpow.mpow_plan_tile_table(hb)
    mpow.mpow_plan_tile_table(hb, [shape] * mpow.TILE_TABLE_LEN)
    try:
        mats, ps = [], []
        for i, n in enumerate((5, 40, 100, 144, 200, 256)):
            for j, bad in enumerate((np.nan, np.inf, -np.inf)):
                A = inputs.gaussian(n, 9300 + 10 * i + j)
                A[(3 * j) % n, (7 + j) % n] = bad
                for p in (2, 3, 17):
                    mats.append(A)
                    ps.append(p)
        pk = Packed(mats)
        run_batch(hb, pk, ps)
        for i, (A, p) in enumerate(zip(mats, ps)):
            Mb, sb = pk.result(i)
            Mp, sp = run_gpu(hp, A, p)
            assert np.array_equal(Mb, Mp, equal_nan=True) and sb == sp, (A.shape[0], p, i)
            assert not np.all(np.isfinite(Mb)), (A.shape[0], p)
    finally:
        mpow.mpow_plan_tile_table(hb, saved)


def test_back_to_back_batches_with_launch_groups(plans):
    # Several batches in flight on one stream (no synchronisation between the
    # calls, so descriptor slots and workers' scratch are reused while earlier
    # batches run), with a table that splits each batch into several launch
    # groups: every call's results equal those of a synchronised call.
    import torch
    hb, _ = plans
    mats, ps = edge_batch(11)
    saved = mpow.mpow_plan_tile_table(hb)
    try:
        mpow.mpow_plan_tile_table(hb, [(b + 1) % 5 for b in range(mpow.TILE_TABLE_LEN)])
        ref = Packed(mats)
        run_batch(hb, ref, ps)
        want = [ref.result(i) for i in range(len(ps))]
        packs = [Packed(mats) for _ in range(4)]
        st = torch.cuda.current_stream().cuda_stream
        print(f"  [gpu] {len(packs)} back-to-back batches of {len(ps)}", flush=True)
        for pk in packs:
            mpow.mpow_run_batched(hb, len(ps), mpow.BatchArgs(pk.a_ptrs, pk.ns, ps, pk.o_ptrs),
                                  log2_scale=pk.scale.data_ptr(), stream=st)
        torch.cuda.synchronize()
        for pk in packs:
            for i in range(len(ps)):
                M, s = pk.result(i)
                assert np.array_equal(M, want[i][0]) and s == want[i][1], i
    finally:
        mpow.mpow_plan_tile_table(hb, saved)
