// C ABI of the library: argument checks, the product schedule of p, plan and
// workspace ownership, and the enqueueing of one power.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "mpow_internal.h"

using namespace mpow;

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

mpow_status device_error(mpow_plan *plan, hipError_t e) {
    if (plan) plan->last_error = (int)e;
    return MPOW_ERR_DEVICE;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace sizes, in bytes, for a plan of max_n.
struct Sizes {
    size_t buf, part, partA, escale, split, desc, scratch, total;
};

constexpr int kWorkersForSizing = 512;  // 256 CUs x 2 resident workers

size_t batch_desc_bytes(int max_batch) {
    return sizeof(BatchHeader) + (size_t)max_batch * sizeof(BatchItem);
}

bool sizes_for(int max_n, int max_batch, int mode, int workers, Sizes *z) {
    if (max_n < 1) return false;
    const size_t n = (size_t)max_n;
    const size_t t32 = (n + 31) / 32;
    z->buf = round_up(n * n * sizeof(float), 256);
    z->part = round_up(t32 * t32 * sizeof(double), 256);
    z->partA = round_up(512 * sizeof(double), 256);
    z->escale = round_up((MPOW_MAX_STEPS + 2) * sizeof(int), 256);
    const size_t ld = (size_t)split_ld(max_n);
    z->split = mode == MPOW_FP32 ? 0 : round_up(ld * ld * 2, 256);  // one 16-bit ld x ld array
    const size_t bmax = (size_t)(max_n < kBatchMaxN ? max_n : kBatchMaxN);
    z->desc = max_batch > 0 ? round_up(batch_desc_bytes(max_batch), 256) : 0;
    z->scratch = max_batch > 0 ? round_up((size_t)workers * 2 * bmax * bmax * sizeof(float), 256) : 0;
    z->total = 2 * z->buf + 2 * z->part + z->partA + z->escale + 8 * z->split + z->desc + z->scratch;
    return true;
}

// [a, a + alen) and [b, b + blen) share at least one byte
bool ranges_overlap(const void *a, size_t alen, const void *b, size_t blen) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + blen && y < x + alen;
}

int popcount64(uint64_t v) { return __builtin_popcountll(v); }

hipEvent_t take_event(mpow_plan *plan) {
    if (!plan->free_events.empty()) {
        hipEvent_t e = plan->free_events.back();
        plan->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

mpow_status record_start(mpow_plan *plan, int kernel, double flop, hipStream_t s, TimingRecord *rec) {
    rec->kernel = kernel;
    rec->flop = flop;
    rec->start = take_event(plan);
    rec->stop = take_event(plan);
    if (!rec->start || !rec->stop) return device_error(plan, hipErrorOutOfMemory);
    const hipError_t e = hipEventRecord(rec->start, s);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

mpow_status record_stop(mpow_plan *plan, TimingRecord *rec, hipStream_t s) {
    const hipError_t e = hipEventRecord(rec->stop, s);
    if (e != hipSuccess) return device_error(plan, e);
    plan->pending.push_back(*rec);
    return MPOW_SUCCESS;
}

// Split-precision power: A is split once (both layouts); after every product
// but the last, the float32 result is split again with its own scale.
mpow_status run_split(mpow_plan *plan, const float *A, int n, int64_t p, const uint8_t *ops, int G,
                      int nbA, float *out, double *log2_scale, hipStream_t s) {
    Workspace &ws = plan->ws;
    const int mode = plan->mode;
    const int ld = split_ld(n);
    const bool timing = (plan->flags & MPOW_FLAG_TIMING) != 0;
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const int kernel = gemm_split_pick(mode, n);
    const int tiles = gemm_split_tiles(kernel, n);

    SplitLaunch sl;
    sl.X = A;
    sl.part = ws.partA;
    sl.nPart = nbA;
    sl.n = n;
    sl.ld = ld;
    sl.hi = ws.sa[0];
    sl.lo = ws.sa[1];
    sl.hiT = ws.sa[2];
    sl.loT = ws.sa[3];
    sl.eSlot = ws.escale;
    hipError_t e = launch_split(mode, sl, s);
    if (e != hipSuccess) return device_error(plan, e);

    for (int k = 1; k <= G; ++k) {
        void *const *xs = (k == 1) ? ws.sa : ws.sx;
        void *const *ys = (ops[k - 1] == 0) ? xs : ws.sa;
        SplitGemmLaunch g;
        g.xh = xs[0];
        g.xl = xs[1];
        g.yh = ys[2];
        g.yl = ys[3];
        g.C = ws.buf[k & 1];
        g.partC = ws.part[k & 1];
        g.n = n;
        g.ld = ld;
        TimingRecord rec{};
        if (timing) {
            const mpow_status st = record_start(plan, kernel, flop, s, &rec);
            if (st != MPOW_SUCCESS) return st;
        }
        e = gemm_split_launch(kernel, g, s);
        if (e != hipSuccess) return device_error(plan, e);
        if (timing) {
            const mpow_status st = record_stop(plan, &rec, s);
            if (st != MPOW_SUCCESS) return st;
        }
        if (k < G) {
            sl.X = g.C;
            sl.part = g.partC;
            sl.nPart = tiles;
            sl.hi = ws.sx[0];
            sl.lo = ws.sx[1];
            sl.hiT = ws.sx[2];
            sl.loT = ws.sx[3];
            sl.eSlot = ws.escale + k;
            e = launch_split(mode, sl, s);
            if (e != hipSuccess) return device_error(plan, e);
        }
    }
    e = launch_finish(ws.buf[G & 1], n, ws.part[G & 1], tiles, ws.escale, p, G, out, log2_scale, s);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

}  // namespace

extern "C" {

const char *mpow_status_str(int status) {
    switch (status) {
        case MPOW_SUCCESS: return "success";
        case MPOW_ERR_INVALID: return "invalid argument";
        case MPOW_ERR_UNSUPPORTED: return "unsupported";
        case MPOW_ERR_NOMEM: return "out of memory";
        case MPOW_ERR_DEVICE: return "device error";
        case MPOW_ERR_BUDGET: return "exceeds memory budget";
        default: return "unknown status";
    }
}

int mpow_gemm_count(int64_t p) {
    if (p < 0) return -1;
    if (p < 2) return 0;
    const int top = 63 - __builtin_clzll((unsigned long long)p);
    return top + popcount64((uint64_t)p) - 1;
}

int mpow_schedule(int64_t p, uint8_t *ops, int cap) {
    const int g = mpow_gemm_count(p);
    if (g < 0) return -1;
    if (g == 0) return 0;
    if (!ops || cap < g) return -1;
    const int top = 63 - __builtin_clzll((unsigned long long)p);
    int k = 0;
    for (int bit = top - 1; bit >= 0; --bit) {
        ops[k++] = 0;
        if ((p >> bit) & 1) ops[k++] = 1;
    }
    return k;
}

size_t mpow_workspace_bytes(int max_n, int max_batch, int mode) {
    Sizes z;
    if (max_batch < 0 || mode < 0 || mode > MPOW_BF16X3 ||
        !sizes_for(max_n, max_batch, mode, kWorkersForSizing, &z))
        return 0;
    return z.total;
}

mpow_status mpow_plan_create(mpow_plan_t *out_plan, int device, int max_n, int max_batch,
                             int mode, uint32_t flags) {
    if (!out_plan) return MPOW_ERR_INVALID;
    *out_plan = nullptr;
    if (max_n < 1 || max_batch < 0 || mode < 0 || mode > MPOW_BF16X3 ||
        (flags & ~(MPOW_FLAG_TIMING | MPOW_FLAG_POISON)) != 0)
        return MPOW_ERR_INVALID;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return MPOW_ERR_DEVICE;
    int workers = 0;
    if (max_batch > 0) {
        DeviceGuard g0(device);
        int cus = 0;
        if (!g0.ok || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) !=
                          hipSuccess)
            return MPOW_ERR_DEVICE;
        workers = cus * batched_occupancy();
        if (workers < 1) workers = 1;
    }
    Sizes z;
    sizes_for(max_n, max_batch, mode, workers, &z);

    mpow_plan *plan = new (std::nothrow) mpow_plan();
    if (!plan) return MPOW_ERR_NOMEM;
    plan->device = device;
    plan->max_n = max_n;
    plan->max_batch = max_batch;
    plan->mode = mode;
    plan->flags = flags;

    DeviceGuard guard(device);
    if (!guard.ok) {
        delete plan;
        return MPOW_ERR_DEVICE;
    }
    char *base = nullptr;
    hipError_t e = hipMalloc((void **)&base, z.total);
    if (e != hipSuccess || !base) {
        (void)hipGetLastError();
        delete plan;
        return MPOW_ERR_NOMEM;
    }
    e = hipMemset(base, (flags & MPOW_FLAG_POISON) ? 0xFF : 0, z.total);
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete plan;
        return MPOW_ERR_DEVICE;
    }
    char *q = base;
    plan->ws.buf[0] = (float *)q; q += z.buf;
    plan->ws.buf[1] = (float *)q; q += z.buf;
    plan->ws.part[0] = (double *)q; q += z.part;
    plan->ws.part[1] = (double *)q; q += z.part;
    plan->ws.partA = (double *)q; q += z.partA;
    plan->ws.escale = (int *)q; q += z.escale;
    for (int k = 0; k < 4 && z.split; ++k) {
        plan->ws.sx[k] = q; q += z.split;
        plan->ws.sa[k] = q; q += z.split;
    }
    if (max_batch > 0) {
        plan->batch_desc = q; q += z.desc;
        plan->batch_scratch = (float *)q; q += z.scratch;
        const int bmax = max_n < kBatchMaxN ? max_n : kBatchMaxN;
        plan->batch_slot_floats = (int64_t)bmax * bmax;
        plan->batch_workers = workers;
        for (int b = 0; b <= kBatchMaxN / 16; ++b) plan->batch_cfg[b] = batched_cfg_for(b * 16);
        bool ok = hipHostMalloc(&plan->batch_host, batch_desc_bytes(max_batch), hipHostMallocDefault) ==
                  hipSuccess;
        ok = ok && hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipEventCreateWithFlags(&plan->batch_done, hipEventDisableTiming) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            if (plan->batch_host) (void)hipHostFree(plan->batch_host);
            if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
            (void)hipFree(base);
            delete plan;
            return MPOW_ERR_NOMEM;
        }
    }
    plan->ws.part_cap = z.part / sizeof(double);
    plan->ws.partA_cap = z.partA / sizeof(double);
    *out_plan = plan;
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_destroy(mpow_plan_t plan) {
    if (!plan) return MPOW_SUCCESS;
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    for (auto &r : plan->pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (auto e : plan->free_events) (void)hipEventDestroy(e);
    if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
    if (plan->batch_done) (void)hipEventDestroy(plan->batch_done);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->batch_host) (void)hipHostFree(plan->batch_host);
    (void)hipFree(plan->ws.buf[0]);
    delete plan;
    return MPOW_SUCCESS;
}

int mpow_last_device_error(mpow_plan_t plan) { return plan ? plan->last_error : 0; }

mpow_status mpow_run(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                     double *log2_scale, void *stream) {
    if (!plan || !A || !out || n < 1 || p < 0) return MPOW_ERR_INVALID;
    if (n > plan->max_n) return MPOW_ERR_INVALID;
    const size_t bytes = (size_t)n * (size_t)n * sizeof(float);
    if ((const void *)A != (const void *)out && ranges_overlap(A, bytes, out, bytes))
        return MPOW_ERR_INVALID;
    if (((uintptr_t)A & 3) || ((uintptr_t)out & 3) || ((uintptr_t)log2_scale & 7))
        return MPOW_ERR_INVALID;
    if (log2_scale && (ranges_overlap(log2_scale, sizeof(double), A, bytes) ||
                       ranges_overlap(log2_scale, sizeof(double), out, bytes)))
        return MPOW_ERR_INVALID;

    hipStream_t s = (hipStream_t)stream;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    Workspace &ws = plan->ws;
    hipError_t e;

    if (p == 0) {
        e = launch_identity(out, n, log2_scale, s);
        return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
    }

    const int nbA = norm_blocks(n);
    e = launch_sumsq(A, n, ws.partA, nbA, s);
    if (e != hipSuccess) return device_error(plan, e);

    uint8_t ops[MPOW_MAX_STEPS];
    const int G = mpow_schedule(p, ops, MPOW_MAX_STEPS);
    if (plan->mode != MPOW_FP32 && G > 0) return run_split(plan, A, n, p, ops, G, nbA, out, log2_scale, s);
    const int kernel = gemm_pick(n);
    const int tiles = gemm_tiles(kernel, n);
    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    const bool timing = (plan->flags & MPOW_FLAG_TIMING) != 0;
    const double flop = 2.0 * (double)n * (double)n * (double)n;

    const float *X = A;
    const double *partX = ws.partA;
    int nPartX = nbA;
    for (int k = 1; k <= G; ++k) {
        GemmLaunch g;
        g.X = X;
        g.partX = partX;
        g.nPartX = nPartX;
        if (ops[k - 1] == 0) {
            g.Y = X;
            g.partY = partX;
            g.nPartY = nPartX;
        } else {
            g.Y = A;
            g.partY = ws.partA;
            g.nPartY = nbA;
        }
        g.C = ws.buf[k & 1];
        g.partC = ws.part[k & 1];
        g.eSlot = ws.escale + (k - 1);
        g.n = n;
        TimingRecord rec{};
        if (timing) {
            rec.kernel = kernel;
            rec.flop = flop;
            rec.start = take_event(plan);
            rec.stop = take_event(plan);
            if (!rec.start || !rec.stop) return device_error(plan, hipErrorOutOfMemory);
            e = hipEventRecord(rec.start, s);
            if (e != hipSuccess) return device_error(plan, e);
        }
        e = gemm_launch(kernel, g, vec4, s);
        if (e != hipSuccess) return device_error(plan, e);
        if (timing) {
            e = hipEventRecord(rec.stop, s);
            if (e != hipSuccess) return device_error(plan, e);
            plan->pending.push_back(rec);
        }
        X = g.C;
        partX = g.partC;
        nPartX = tiles;
    }

    e = launch_finish(X, n, partX, nPartX, ws.escale, p, G, out, log2_scale, s);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

mpow_status mpow_run_batched(mpow_plan_t plan, int count, const float *const *A, const int *n,
                             const int64_t *p, float *const *out, double *log2_scale,
                             void *stream) {
    if (!plan || count < 0 || count > plan->max_batch) return MPOW_ERR_INVALID;
    if (count > 0 && (!A || !n || !p || !out)) return MPOW_ERR_INVALID;
    if ((uintptr_t)log2_scale & 7) return MPOW_ERR_INVALID;
    for (int i = 0; i < count; ++i) {
        const int ni = n[i];
        if (!A[i] || !out[i] || ni < 1 || ni > plan->max_n || ni > kBatchMaxN || p[i] < 0)
            return MPOW_ERR_INVALID;
        if (((uintptr_t)A[i] & 3) || ((uintptr_t)out[i] & 3)) return MPOW_ERR_INVALID;
        const size_t bytes = (size_t)ni * (size_t)ni * sizeof(float);
        if ((const void *)A[i] != (const void *)out[i] && ranges_overlap(A[i], bytes, out[i], bytes))
            return MPOW_ERR_INVALID;
    }
    if (count == 0) return MPOW_SUCCESS;
    if (plan->mode != MPOW_FP32) return MPOW_ERR_UNSUPPORTED;

    hipStream_t s = (hipStream_t)stream;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    hipError_t e;
    // The graph's copy reads the pinned descriptors: wait until the previous
    // batch's copy has consumed them before rewriting.
    if (plan->batch_pending) {
        e = hipEventSynchronize(plan->batch_done);
        if (e != hipSuccess) return device_error(plan, e);
        plan->batch_pending = false;
    }

    // Longest work first: estimated work G(p) * n^3, ties by input order.
    std::vector<int> order(count);
    std::vector<double> work(count);
    for (int i = 0; i < count; ++i) {
        order[i] = i;
        const double nn = (double)n[i];
        work[i] = (double)(mpow_gemm_count(p[i]) + 1) * nn * nn * nn;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    BatchHeader *hdr = (BatchHeader *)plan->batch_host;
    hdr->counter = 0;
    hdr->count = count;
    hdr->pad[0] = hdr->pad[1] = 0;
    BatchItem *items = (BatchItem *)(hdr + 1);
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        items[k].A = A[i];
        items[k].out = out[i];
        items[k].scale = log2_scale ? log2_scale + i : nullptr;
        items[k].p = p[i];
        items[k].n = n[i];
        items[k].cfg = plan->batch_cfg[(n[i] + 15) / 16];
    }

    if (!plan->graph_exec || plan->graph_count != count) {
        if (plan->graph_exec) {
            (void)hipGraphExecDestroy(plan->graph_exec);
            plan->graph_exec = nullptr;
        }
        BatchLaunch bl;
        bl.desc = plan->batch_desc;
        bl.scratch = plan->batch_scratch;
        bl.slot_floats = plan->batch_slot_floats;
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return device_error(plan, e);
        const hipError_t e1 = hipMemcpyAsync(plan->batch_desc, plan->batch_host,
                                             batch_desc_bytes(count), hipMemcpyHostToDevice,
                                             plan->capture_stream);
        const hipError_t e2 = launch_batched(bl, plan->batch_workers, plan->capture_stream);
        e = hipStreamEndCapture(plan->capture_stream, &graph);
        if (e1 != hipSuccess || e2 != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return device_error(plan, e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e));
        }
        e = hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plan->graph_exec = nullptr;
            return device_error(plan, e);
        }
        plan->graph_count = count;
    }
    e = hipGraphLaunch(plan->graph_exec, s);
    if (e != hipSuccess) return device_error(plan, e);
    e = hipEventRecord(plan->batch_done, s);
    if (e != hipSuccess) return device_error(plan, e);
    plan->batch_pending = true;
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_timing(mpow_plan_t plan, int kernel, int64_t *launches, double *total_ms,
                             double *total_flop, const char **name) {
    if (!plan || !(plan->flags & MPOW_FLAG_TIMING) || kernel < 0 || kernel >= MPOW_KERNEL_COUNT)
        return MPOW_ERR_INVALID;
    DeviceGuard guard(plan->device);
    for (auto &r : plan->pending) {
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return device_error(plan, e);
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess) return device_error(plan, e);
        plan->launches[r.kernel] += 1;
        plan->ms[r.kernel] += ms;
        plan->flop[r.kernel] += r.flop;
        plan->free_events.push_back(r.start);
        plan->free_events.push_back(r.stop);
    }
    plan->pending.clear();
    if (launches) *launches = plan->launches[kernel];
    if (total_ms) *total_ms = plan->ms[kernel];
    if (total_flop) *total_flop = plan->flop[kernel];
    if (name) *name = gemm_name(kernel) ? gemm_name(kernel) : gemm_split_name(kernel);
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_timing_reset(mpow_plan_t plan) {
    if (!plan) return MPOW_ERR_INVALID;
    int64_t l;
    double m, f;
    mpow_status st = MPOW_SUCCESS;
    if (plan->flags & MPOW_FLAG_TIMING) st = mpow_plan_timing(plan, 0, &l, &m, &f, nullptr);
    for (int k = 0; k < MPOW_KERNEL_COUNT; ++k) {
        plan->launches[k] = 0;
        plan->ms[k] = 0.0;
        plan->flop[k] = 0.0;
    }
    return st;
}

}  // extern "C"
