// Host runtime: workspace layout, the enqueueing of one power (the product
// schedule of the paper's section 4.3 method), ragged-batch contexts and
// HIP-event timing.  Shared by plans and by the request server.
#include <algorithm>
#include <vector>

#include "mpow_internal.h"

namespace mpow {

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

namespace {

struct Layout {
    size_t buf, part, partA, escale, split, total;
};

Layout layout_for(int max_n, int mode) {
    Layout z;
    z.buf = ws_buf_bytes(max_n);
    z.part = ws_part_bytes(max_n);
    z.partA = ws_partA_bytes();
    z.escale = ws_escale_bytes();
    const size_t ld = (size_t)split_ld(max_n);
    z.split = mode == MPOW_FP32 ? 0 : round_up(ld * ld * 2, 256);
    // two operands (running matrix, A) x two layouts x the mode's parts, and
    // for the fused split a second set of the running matrix's
    const int sets = split_fused(mode) ? 6 : 4;
    z.total = 2 * z.buf + 2 * z.part + z.partA + z.escale + sets * split_parts(mode) * z.split;
    return z;
}

}  // namespace

size_t workspace_bytes(int max_n, int mode) { return layout_for(max_n, mode).total; }

void workspace_carve(char *base, int max_n, int mode, Workspace *ws) {
    const Layout z = layout_for(max_n, mode);
    char *q = base;
    ws->buf[0] = (float *)q; q += z.buf;
    ws->buf[1] = (float *)q; q += z.buf;
    ws->part[0] = (double *)q; q += z.part;
    ws->part[1] = (double *)q; q += z.part;
    ws->partA = (double *)q; q += z.partA;
    ws->escale = (int *)q; q += z.escale;
    for (int l = 0; l < 2; ++l)
        for (int k = 0; k < split_parts(mode); ++k) {
            ws->sx[l][k] = (void *)q; q += z.split;
            ws->sa[l][k] = (void *)q; q += z.split;
            if (split_fused(mode)) {
                ws->sy[l][k] = (void *)q;
                q += z.split;
            }
        }
    ws->max_n = max_n;
    ws->mode = mode;
}

// ---------------------------------------------------------------- timing

hipError_t TimingSink::start(int kernel, double f, hipStream_t s, TimingRecord *rec) {
    rec->kernel = kernel;
    rec->flop = f;
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (!free_events.empty()) {
            ev[i] = free_events.back();
            free_events.pop_back();
        } else {
            const hipError_t e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) return e;
        }
    }
    rec->start = ev[0];
    rec->stop = ev[1];
    return hipEventRecord(rec->start, s);
}

hipError_t TimingSink::stop(TimingRecord *rec, hipStream_t s) {
    const hipError_t e = hipEventRecord(rec->stop, s);
    if (e == hipSuccess) pending.push_back(*rec);
    return e;
}

hipError_t TimingSink::collect() {
    for (auto &r : pending) {
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return e;
        float t = 0.f;
        e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) return e;
        launches[r.kernel] += 1;
        ms[r.kernel] += t;
        flop[r.kernel] += r.flop;
        free_events.push_back(r.start);
        free_events.push_back(r.stop);
    }
    pending.clear();
    return hipSuccess;
}

void TimingSink::reset() {
    for (int k = 0; k < MPOW_KERNEL_COUNT; ++k) {
        launches[k] = 0;
        ms[k] = 0.0;
        flop[k] = 0.0;
    }
}

void TimingSink::destroy() {
    for (auto &r : pending) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    pending.clear();
    for (auto e : free_events) (void)hipEventDestroy(e);
    free_events.clear();
}

// ---------------------------------------------------------------- one power

// Left-to-right sliding-window schedule with windows of up to w bits (w = 1
// is binary exponentiation).  The bits of p are read from the top; a zero
// bit squares the running matrix R, and a window (a run of at most w bits
// that starts and ends with a one, value v) squares R once per bit and then
// multiplies it by the precomputed odd power A^v.  The first window sets R
// to A^v itself.  The odd powers up to the largest v used are precomputed
// as A^2 = A.A, A^3 = A.A^2, A^5 = A^3.A^2, ...  Slots: kSlotA, kSlotA2,
// A^(2i+1) at kSlotA2 + i, and R alternating between kSlotR0 and kSlotR1.
int window_schedule(int64_t p, int w, uint8_t *ops, int cap, int *result) {
    if (p < 1 || w < 1 || w > 3) return -1;
    const int top = 63 - __builtin_clzll((unsigned long long)p);
    // windows, top down: len = bits covered, v = 0 for a lone zero bit
    int wlen[64], wval[64], nw = 0, maxv = 1;
    for (int i = top; i >= 0;) {
        if (!((p >> i) & 1)) {
            wlen[nw] = 1;
            wval[nw++] = 0;
            --i;
            continue;
        }
        int j = i - w + 1 < 0 ? 0 : i - w + 1;
        while (!((p >> j) & 1)) ++j;
        const int v = (int)((p >> j) & ((1ll << (i - j + 1)) - 1));
        wlen[nw] = i - j + 1;
        wval[nw++] = v;
        maxv = v > maxv ? v : maxv;
        i = j - 1;
    }
    int k = 0;
    auto emit = [&](int dst, int x, int y) -> bool {
        if (ops) {
            if (k >= cap) return false;
            ops[3 * k] = (uint8_t)dst;
            ops[3 * k + 1] = (uint8_t)x;
            ops[3 * k + 2] = (uint8_t)y;
        }
        ++k;
        return true;
    };
    auto slot_of = [](int v) { return v == 1 ? kSlotA : kSlotA2 + (v - 1) / 2; };
    if (maxv >= 3) {
        if (!emit(kSlotA2, kSlotA, kSlotA)) return -1;
        for (int v = 3; v <= maxv; v += 2)
            if (!emit(slot_of(v), slot_of(v - 2), kSlotA2)) return -1;
    }
    int R = slot_of(wval[0]);
    auto next_r = [&]() { return R == kSlotR0 ? kSlotR1 : kSlotR0; };
    for (int q = 1; q < nw; ++q) {
        for (int s = 0; s < wlen[q]; ++s) {
            const int d = next_r();
            if (!emit(d, R, R)) return -1;
            R = d;
        }
        if (wval[q]) {
            const int d = next_r();
            if (!emit(d, R, slot_of(wval[q]))) return -1;
            R = d;
        }
    }
    *result = R;
    return k;
}

int ws_product_kernel(const Workspace &ws, int n, bool vec4) {
    if (ws.kernel >= 0) return ws.kernel;
    const int b = (n + 255) / 256;
    if (ws.mode == MPOW_FP32) {
        // tuned picks are among the LDS-DMA tiles (16-byte loads) from n = 768
        if (vec4 && n >= 768 && b < kPickBuckets && ws.pick1[b] > 0) return ws.pick1[b] - 1;
        return gemm_pick(n, vec4);
    }
    if (b < kPickBuckets && ws.pick1[b] > 0) return ws.pick1[b] - 1;
    return gemm_split_pick(ws.mode, n);
}

namespace {

int schedule_of(int64_t p, uint8_t *ops) {
    if (p < 2) return 0;
    const int top = 63 - __builtin_clzll((unsigned long long)p);
    int k = 0;
    for (int bit = top - 1; bit >= 0; --bit) {
        ops[k++] = 0;
        if ((p >> bit) & 1) ops[k++] = 1;
    }
    return k;
}

#define MPOW_TRY(expr)                          \
    do {                                        \
        const hipError_t e_ = (expr);           \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// Float32 products: step k computes C_k = (2^-e X)(2^-e' Y) from the
// partial sums of its operands; X = C_{k-1} (C_0 = A), Y = X (square) or A.
// The first step is always A^2, whose launch records e_A in the first
// exponent slot; the multiplies read e_A from there rather than reducing A's
// partial sums again (one device load instead of a workgroup-wide reduction
// of hundreds of partials, whose latency every workgroup of a small product
// pays).
//
// For small n on the whole-K 32 x 32 kernels the first product reduces the
// input's norm itself (every workgroup reads the n^2 inputs once more), so
// the power needs no separate norm launch before it: a dependent launch
// costs a few microseconds, about what a whole small product takes.
static bool fp32_norm_in_kernel(const Workspace &ws, const float *A, int n) {
    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    const int kernel = gemm_resolve(ws_product_kernel(ws, n, vec4), n, vec4);
    return vec4 && n <= kNormInKernelMaxN &&
           (kernel == MPOW_KERNEL_GEMM_F32_32_K4_DMA || kernel == MPOW_KERNEL_GEMM_F32_32_K8_DMA);
}

hipError_t run_fp32(const Workspace &ws, const float *A, int n, int64_t p, const uint8_t *ops,
                    int G, int nbA, bool normInKernel, float *out, double *log2_scale,
                    hipStream_t s, TimingSink *timing) {
    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    int kernel = ws_product_kernel(ws, n, vec4);
    kernel = gemm_resolve(kernel, n, vec4);
    const int tiles = gemm_tiles(kernel, n);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const float *X = A;
    const double *partX = normInKernel ? nullptr : ws.partA;
    int nPartX = normInKernel ? 0 : nbA;
    for (int k = 1; k <= G; ++k) {
        GemmLaunch g;
        g.X = X;
        g.partX = partX;
        g.nPartX = nPartX;
        if (k == 1 && normInKernel) g.normA = A;  // A^2: both operands are A
        if (ops[k - 1] == 0) {
            g.Y = X;
            g.partY = partX;
            g.nPartY = nPartX;
        } else {
            g.Y = A;
            g.partY = nullptr;
            g.nPartY = 0;
            g.eYin = ws.escale;  // e_A, recorded by step 1 (A^2)
        }
        g.C = ws.buf[k & 1];
        g.partC = ws.part[k & 1];
        g.eSlot = ws.escale + (k - 1);
        g.n = n;
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(kernel, flop, s, &rec));
        MPOW_TRY(gemm_launch(kernel, g, vec4, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
        X = g.C;
        partX = g.partC;
        nPartX = tiles;
    }
    return launch_finish(X, n, partX, nPartX, ws.escale, p, out, log2_scale, s);
}

// Split-precision products: A is split once (both layouts).  FP16X3: after
// every product but the last, the float32 result is split again with its own
// scale (the FP16 parts need the scale before rounding).  BF16 modes: every
// product but the last writes the parts of its unnormalised result itself
// (BF16 keeps float32's exponent range, so rounding the unscaled value and
// scaling afterwards by an exact power of two give the same parts), with its
// partial sums; the next product derives the exponent from those and scales
// its sums by 2^-(eX + eY) in its epilogue.
hipError_t run_split_fused(const Workspace &ws, int n, const uint8_t *ops, int G, int kernel,
                           float *out, double *log2_scale, hipStream_t s, TimingSink *timing,
                           int64_t p) {
    const int np = split_parts(ws.mode);
    const int ld = split_ld(n);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const int tiles = gemm_split_tiles(kernel, n);
    void *const(*cur)[3] = ws.sa;  // the left operand's parts
    const double *partX = nullptr;  // null: parts of a normalised matrix
    int nPartX = 0;
    for (int k = 1; k <= G; ++k) {
        const bool sq = ops[k - 1] == 0;
        SplitGemmLaunch g{};
        for (int q = 0; q < np; ++q) {
            g.x[q] = cur[0][q];
            g.y[q] = sq ? cur[1][q] : ws.sa[1][q];
        }
        g.partX = partX;
        g.nPartX = nPartX;
        g.partY = sq ? partX : nullptr;
        g.nPartY = sq ? nPartX : 0;
        g.eSlot = k > 1 ? ws.escale + (k - 1) : nullptr;
        g.partC = ws.part[k & 1];
        g.n = n;
        g.ld = ld;
        void *const(*dest)[3] = cur == ws.sx ? ws.sy : ws.sx;
        if (k < G) {
            for (int q = 0; q < np; ++q) {
                g.prm[q] = dest[0][q];
                g.ptr[q] = dest[1][q];
            }
        } else {
            g.C = ws.buf[G & 1];
        }
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(kernel, flop, s, &rec));
        MPOW_TRY(gemm_split_launch(kernel, g, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
        cur = dest;
        partX = g.partC;
        nPartX = tiles;
    }
    return launch_finish(ws.buf[G & 1], n, ws.part[G & 1], tiles, ws.escale, p, out, log2_scale, s);
}

hipError_t run_split(const Workspace &ws, const float *A, int n, int64_t p, const uint8_t *ops,
                     int G, int nbA, float *out, double *log2_scale, hipStream_t s,
                     TimingSink *timing) {
    const int mode = ws.mode;
    const int ld = split_ld(n);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const int kernel = ws_product_kernel(ws, n, false);
    const int tiles = gemm_split_tiles(kernel, n);

    const int np = split_parts(mode);
    SplitLaunch sl{};
    sl.X = A;
    sl.part = ws.partA;
    sl.nPart = nbA;
    sl.n = n;
    sl.ld = ld;
    for (int k = 0; k < np; ++k) {
        sl.rm[k] = ws.sa[0][k];
        sl.tr[k] = ws.sa[1][k];
    }
    sl.eSlot = ws.escale;
    MPOW_TRY(launch_split(mode, sl, s));
    if (split_fused(mode) && !ws.split_pass)
        return run_split_fused(ws, n, ops, G, kernel, out, log2_scale, s, timing, p);

    for (int k = 1; k <= G; ++k) {
        void *const(*xs)[3] = (k == 1) ? ws.sa : ws.sx;
        void *const(*ys)[3] = (ops[k - 1] == 0) ? xs : ws.sa;
        SplitGemmLaunch g{};
        for (int q = 0; q < np; ++q) {
            g.x[q] = xs[0][q];
            g.y[q] = ys[1][q];
        }
        g.C = ws.buf[k & 1];
        g.partC = ws.part[k & 1];
        g.n = n;
        g.ld = ld;
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(kernel, flop, s, &rec));
        MPOW_TRY(gemm_split_launch(kernel, g, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
        if (k < G) {
            sl.X = g.C;
            sl.part = g.partC;
            sl.nPart = tiles;
            for (int q = 0; q < np; ++q) {
                sl.rm[q] = ws.sx[0][q];
                sl.tr[q] = ws.sx[1][q];
            }
            sl.eSlot = ws.escale + k;
            MPOW_TRY(launch_split(mode, sl, s));
        }
    }
    return launch_finish(ws.buf[G & 1], n, ws.part[G & 1], tiles, ws.escale, p, out, log2_scale, s);
}

// Float32 products along a window schedule (ops from window_schedule, G >= 1).
hipError_t run_fp32_window(const Workspace &ws, const float *A, int n, const uint8_t *ops,
                           int G, int result, int nbA, float *out, double *log2_scale,
                           hipStream_t s, TimingSink *timing) {
    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    int kernel = ws_product_kernel(ws, n, vec4);
    kernel = gemm_resolve(kernel, n, vec4);
    const int tiles = gemm_tiles(kernel, n);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const float *mat[kSlots] = {A, ws.wp[0], ws.wp[1], ws.wp[2], ws.wp[3], ws.buf[0], ws.buf[1]};
    double *part[kSlots] = {ws.partA, ws.wpart[0], ws.wpart[1], ws.wpart[2], ws.wpart[3],
                            ws.part[0], ws.part[1]};
    int npart[kSlots];
    for (int i = 0; i < kSlots; ++i) npart[i] = i == kSlotA ? nbA : tiles;
    GraphOps g{};
    g.count = G;
    g.result = result;
    for (int k = 0; k < G; ++k) {
        const int d = ops[3 * k], x = ops[3 * k + 1], y = ops[3 * k + 2];
        g.op[k][0] = (uint8_t)d;
        g.op[k][1] = (uint8_t)x;
        g.op[k][2] = (uint8_t)y;
        GemmLaunch L{};
        L.X = mat[x];
        L.partX = part[x];
        L.nPartX = npart[x];
        L.Y = mat[y];
        L.partY = part[y];
        L.nPartY = npart[y];
        L.C = const_cast<float *>(mat[d]);
        L.partC = part[d];
        L.eSlot = ws.escale + k;
        L.eSlotY = ws.escaleY + k;
        L.n = n;
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(kernel, flop, s, &rec));
        MPOW_TRY(gemm_launch(kernel, L, vec4, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
    }
    return launch_finish_graph(mat[result], n, part[result], npart[result], ws.escale, ws.escaleY,
                               g, out, log2_scale, s);
}

}  // namespace

hipError_t enqueue_power(const Workspace &ws, const float *A, int n, int64_t p, float *out,
                         double *log2_scale, hipStream_t s, TimingSink *timing) {
    if (p == 0) return launch_identity(out, n, log2_scale, s);
    // a window schedule (plans that hold one), when it takes fewer products
    // than binary
    int bw = 1;
    if (ws.mode == MPOW_FP32 && ws.escaleY && p >= 2) {
        int best = mpow_gemm_count(p), result = 0;
        for (int w = 2; w <= 3; ++w) {
            const int gw = window_schedule(p, w, nullptr, 0, &result);
            if (gw >= 0 && gw < best) {
                best = gw;
                bw = w;
            }
        }
    }
    if (ws.mode == MPOW_FP32 && bw == 1 && n <= kPowerWgMaxN &&
        (ws.kernel == MPOW_KERNEL_POWER_WG || (ws.kernel < 0 && n <= kPowerWgAutoMaxN))) {
        // the whole power in one workgroup, operands resident in LDS
        uint8_t ops[MPOW_MAX_STEPS];
        const double flop = 2.0 * (double)n * (double)n * (double)n * schedule_of(p, ops);
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(MPOW_KERNEL_POWER_WG, flop, s, &rec));
        MPOW_TRY(launch_power_wg(A, n, p, out, log2_scale, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
        return hipSuccess;
    }
    const int nbA = norm_blocks(n);
    uint8_t ops[MPOW_MAX_STEPS];
    const int G = schedule_of(p, ops);
    const bool normInKernel =
        ws.mode == MPOW_FP32 && bw == 1 && G > 0 && fp32_norm_in_kernel(ws, A, n);
    if (!normInKernel) MPOW_TRY(launch_sumsq(A, n, ws.partA, nbA, s));
    if (G == 0) return launch_finish(A, n, ws.partA, nbA, ws.escale, p, out, log2_scale, s);
    if (ws.mode != MPOW_FP32) return run_split(ws, A, n, p, ops, G, nbA, out, log2_scale, s, timing);
    if (bw > 1) {
        uint8_t wops[3 * kMaxGraphOps];
        int result = 0;
        const int gw = window_schedule(p, bw, wops, kMaxGraphOps, &result);
        if (gw > 0) return run_fp32_window(ws, A, n, wops, gw, result, nbA, out, log2_scale, s, timing);
    }
    return run_fp32(ws, A, n, p, ops, G, nbA, normInKernel, out, log2_scale, s, timing);
}

hipError_t enqueue_power_naive(const Workspace &ws, const float *A, int n, int64_t p, float *out,
                               double *log2_scale, hipStream_t s, TimingSink *timing) {
    if (p == 0) return launch_identity(out, n, log2_scale, s);
    const int nbA = norm_blocks(n);
    MPOW_TRY(launch_sumsq(A, n, ws.partA, nbA, s));
    if (p == 1) return launch_finish(A, n, ws.partA, nbA, ws.escale, p, out, log2_scale, s);
    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    int kernel = ws_product_kernel(ws, n, vec4);
    kernel = gemm_resolve(kernel, n, vec4);
    const int tiles = gemm_tiles(kernel, n);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const int G = (int)(p - 1);
    const float *X = A;
    const double *partX = ws.partA;
    int nPartX = nbA;
    for (int k = 1; k <= G; ++k) {
        GemmLaunch g;
        g.X = X;
        g.partX = partX;
        g.nPartX = nPartX;
        g.Y = A;
        g.partY = ws.partA;
        g.nPartY = nbA;
        g.C = ws.buf[k & 1];
        g.partC = ws.part[k & 1];
        g.eSlot = ws.escale + (k - 1);
        g.n = n;
        TimingRecord rec{};
        if (timing) MPOW_TRY(timing->start(kernel, flop, s, &rec));
        MPOW_TRY(gemm_launch(kernel, g, vec4, s));
        if (timing) MPOW_TRY(timing->stop(&rec, s));
        X = g.C;
        partX = g.partC;
        nPartX = tiles;
    }
    return launch_finish(X, n, partX, nPartX, ws.escale, p, out, log2_scale, s, G);
}

// ---------------------------------------------------------------- ragged batch

size_t batch_desc_bytes(int max_batch) {
    return sizeof(BatchHeader) + (size_t)max_batch * sizeof(BatchItem);
}

// Floats per per-worker scratch buffer: the square of bmax rounded up to a
// multiple of 32 (the whole-power instance pads its matrices so), rounded up
// to 64 floats, so that every buffer starts 256-byte aligned.
static int64_t batch_slot_floats(int bmax) {
    const size_t np = ((size_t)bmax + 31) / 32 * 32;
    return (int64_t)round_up(np * np, 64);
}

size_t batch_device_bytes(int max_batch, int bmax, int workers) {
    return 2 * round_up(batch_desc_bytes(max_batch), 256) +
           round_up((size_t)workers * 2 * (size_t)batch_slot_floats(bmax) * sizeof(float), 256);
}

bool batch_workers_for(int device, int workers[kBatchInstances]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus < 1)
        return false;
    for (int i = 0; i < kBatchInstances; ++i) workers[i] = cus * batched_occupancy(i);
    return true;
}

hipError_t batch_context_init(BatchContext *bc, char *dev, int max_batch, int bmax,
                              const int workers[kBatchInstances]) {
    const size_t desc = round_up(batch_desc_bytes(max_batch), 256);
    bc->slot[0].desc = dev;
    bc->slot[1].desc = dev + desc;
    bc->scratch = (float *)(dev + 2 * desc);
    bc->slot_floats = batch_slot_floats(bmax);
    for (int i = 0; i < kBatchInstances; ++i) bc->workers[i] = workers[i];
    bc->max_batch = max_batch;
    for (int b = 0; b < kTileBuckets; ++b) bc->cfg[b] = batched_cfg_for(b * 16);
    for (int k = 0; k < 2; ++k) {
        MPOW_TRY(hipHostMalloc(&bc->slot[k].host, batch_desc_bytes(max_batch), hipHostMallocDefault));
        MPOW_TRY(hipEventCreateWithFlags(&bc->slot[k].done, hipEventDisableTiming));
    }
    MPOW_TRY(hipStreamCreateWithFlags(&bc->capture_stream, hipStreamNonBlocking));
    return hipSuccess;
}

void batch_context_release(BatchContext *bc) {
    for (int k = 0; k < 2; ++k) {
        BatchSlot &sl = bc->slot[k];
        if (sl.graph_exec) (void)hipGraphExecDestroy(sl.graph_exec);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    if (bc->capture_stream) (void)hipStreamDestroy(bc->capture_stream);

    *bc = BatchContext();
}

hipError_t batch_wait_all(BatchContext *bc) {
    for (int k = 0; k < 2; ++k) {
        BatchSlot &sl = bc->slot[k];
        if (!sl.pending) continue;
        MPOW_TRY(hipEventSynchronize(sl.done));
        sl.pending = false;
    }
    return hipSuccess;
}

int batch_instance(int need, bool all_vec) {
    // the LDS-DMA instance replaces the 128x128 + 64x64 one when every matrix
    // allows 16-byte loads
    return (need == 1 && all_vec) ? 3 : need;
}

int batch_scratch_workers(const int workers[kBatchInstances]) {
    int w = 0;
    for (int i = 0; i < kBatchInstances; ++i)
        if (batched_uses_scratch(i) && workers[i] > w) w = workers[i];
    return w;
}

// Launch group of a matrix and the instance each group runs on: group 0 the
// tiled shapes (on the smallest tiled instance that holds them all), 1 the
// resident form at n <= 64 (instance 4), 2 the resident form at n <= 128
// (5), 3 streamed panels at n > 128 (6), 4 streamed panels at n <= 128 (7).
static int batch_group_of(int cfg, int n) {
    if (cfg == 3) return n <= 64 ? 1 : (n <= 128 ? 2 : 3);
    if (cfg == 4) return n <= 128 ? 4 : 3;
    return 0;
}
constexpr int kGroupInst[kBatchGroups] = {-1, 4, 5, 6, 7};

hipError_t batch_enqueue(BatchContext *bc, int count, const float *const *A, const int *n,
                         const int64_t *p, float *const *out, double *const *scale,
                         hipStream_t s, bool use_graph, hipEvent_t *done) {
    BatchSlot &sl = bc->slot[bc->next];
    // The slot's previous batch must have consumed its descriptors.
    if (sl.pending) {
        MPOW_TRY(hipEventSynchronize(sl.done));
        sl.pending = false;
    }
    // Matrices are grouped by the kernel instance that runs them (one launch
    // per group) and, within a group, taken longest work first: estimated
    // work (G(p) + 1) n^3, ties by input order.
    std::vector<int> order(count), grp(count);
    std::vector<double> work(count);
    uint8_t ops[MPOW_MAX_STEPS];
    int need = 0;  // the smallest tiled instance that holds every tiled matrix's shape
    bool all_vec = true;
    for (int i = 0; i < count; ++i) {
        order[i] = i;
        const double nn = (double)n[i];
        work[i] = (double)(schedule_of(p[i], ops) + 1) * nn * nn * nn;
        const int c = bc->cfg[(n[i] + 15) / 16];
        grp[i] = batch_group_of(c, n[i]);
        if (grp[i] == 0) {
            const int nk = c == 2 ? 2 : (c == 0 ? 1 : 0);
            need = nk > need ? nk : need;
            all_vec = all_vec && n[i] % 4 == 0 && ((uintptr_t)A[i] & 15) == 0;
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return grp[a] != grp[b] ? grp[a] < grp[b] : work[a] > work[b];
    });
    BatchHeader *hdr = (BatchHeader *)sl.host;
    *hdr = BatchHeader();
    hdr->count = count;
    BatchItem *items = (BatchItem *)(hdr + 1);
    for (int g = 0; g < kBatchGroups; ++g) hdr->begin[g] = hdr->end[g] = 0;
    for (int k = 0; k < count; ++k) {
        const int i = order[k];
        items[k].A = A[i];
        items[k].out = out[i];
        items[k].scale = scale ? scale[i] : nullptr;
        items[k].p = p[i];
        items[k].n = n[i];
        items[k].cfg = bc->cfg[(n[i] + 15) / 16];
        const int g = grp[i];
        if (hdr->end[g] == hdr->begin[g]) hdr->begin[g] = k;
        hdr->end[g] = k + 1;
    }
    double gwork[kBatchGroups] = {};
    for (int i = 0; i < count; ++i) gwork[grp[i]] += work[i];
    int inst[kBatchGroups];
    for (int g = 0; g < kBatchGroups; ++g) {
        if (hdr->end[g] == hdr->begin[g])
            inst[g] = -1;
        else if (g == 0)
            inst[g] = batch_instance(need, all_vec);
        else
            inst[g] = kGroupInst[g];
    }
    // Batches share the workers' scratch: order this one after the previous
    // one even when it was enqueued on another stream.
    if (bc->last >= 0 && bc->slot[bc->last].pending)
        MPOW_TRY(hipStreamWaitEvent(s, bc->slot[bc->last].done, 0));
    BatchLaunch bl;
    bl.desc = sl.desc;
    bl.scratch = bc->scratch;
    bl.slot_floats = bc->slot_floats;
    // One persistent launch per group, in order on the stream, the group with
    // the most estimated work first; each starts when the one before has
    // drained (they share the workers' scratch).
    int ord[kBatchGroups], ng = 0;
    for (int g = 0; g < kBatchGroups; ++g)
        if (inst[g] >= 0) ord[ng++] = g;
    std::stable_sort(ord, ord + ng, [&](int a, int b) { return gwork[a] > gwork[b]; });
    auto launch_all = [&](hipStream_t st) -> hipError_t {
        for (int k = 0; k < ng; ++k) {
            bl.group = ord[k];
            const hipError_t e = launch_batched(bl, bc->workers[inst[ord[k]]], inst[ord[k]], st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    bool same = sl.graph_exec && sl.graph_count == count;
    for (int g = 0; g < kBatchGroups; ++g) same = same && sl.graph_inst[g] == inst[g];
    if (use_graph) {
        if (!same) {
            if (sl.graph_exec) {
                (void)hipGraphExecDestroy(sl.graph_exec);
                sl.graph_exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            MPOW_TRY(hipStreamBeginCapture(bc->capture_stream, hipStreamCaptureModeRelaxed));
            const hipError_t e1 = hipMemcpyAsync(sl.desc, sl.host, batch_desc_bytes(count),
                                                 hipMemcpyHostToDevice, bc->capture_stream);
            const hipError_t e2 = e1 == hipSuccess ? launch_all(bc->capture_stream) : hipSuccess;
            const hipError_t e3 = hipStreamEndCapture(bc->capture_stream, &graph);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3);
            }
            const hipError_t e4 = hipGraphInstantiate(&sl.graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e4 != hipSuccess) {
                sl.graph_exec = nullptr;
                return e4;
            }
            sl.graph_count = count;
            for (int g = 0; g < kBatchGroups; ++g) sl.graph_inst[g] = inst[g];
        }
        MPOW_TRY(hipGraphLaunch(sl.graph_exec, s));
    } else {
        MPOW_TRY(hipMemcpyAsync(sl.desc, sl.host, batch_desc_bytes(count), hipMemcpyHostToDevice, s));
        MPOW_TRY(launch_all(s));
    }
    MPOW_TRY(hipEventRecord(sl.done, s));
    sl.pending = true;
    if (done) *done = sl.done;
    bc->last = bc->next;
    bc->next ^= 1;
    return hipSuccess;
}

}  // namespace mpow
