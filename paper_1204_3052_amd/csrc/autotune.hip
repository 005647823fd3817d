// Autotuner.  The paper chose its tile size per problem and per amount of
// local memory by hand (section 4.3.7); here the choices are measured on the
// device:
//  - the ragged-batch kernel's tile table (float32 plans with batch
//    support): for every size bucket each tile shape is timed on a uniform
//    batch that keeps all workers busy, then whole tables on a ragged batch;
//  - the single-matrix product kernel per 256-wide size bucket (every plan):
//    each candidate tile of the plan's mode is timed on one product.
// Every candidate adds each output's products in the same order, so tuning
// changes speed only, never a result.  Timing starts after a warm-up of a
// few tenths of a second (an idle GPU's clock ramps up under load), and the
// candidates of one choice are timed round-robin, each keeping its fastest
// run, so that none is favoured by its place in the order.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mpow_internal.h"

using namespace mpow;

namespace {

constexpr int kBuckets = kTileBuckets;
constexpr int kShapes = kBatchShapes;  // tile shape ids of the batched kernel, all timed
constexpr int64_t kTuneP = 100;        // power of the timing batches (8 products)
static_assert(2 + kShapes <= 8, "Timer::fastest holds at most eight candidates");
constexpr int kPickMaxN = 256 * (kPickBuckets - 1);  // largest size with a tuned pick

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

std::string device_key(int device, int mode) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + " cus=" + std::to_string(prop.multiProcessorCount) + " mode=" + std::to_string(mode);
}

// Single-matrix product candidates of a mode (within a mode they add each
// output's products in the same order).
int pick_candidates(int mode, int *ids) {
    switch (mode) {
        case MPOW_FP32:
            ids[0] = MPOW_KERNEL_GEMM_F32_256x128_DMA;
            ids[1] = MPOW_KERNEL_GEMM_F32_256;
            ids[2] = MPOW_KERNEL_GEMM_F32_128_DMA;
            ids[3] = MPOW_KERNEL_GEMM_F32_64_DMA;
            return 4;
        case MPOW_FP16X3:
            ids[0] = MPOW_KERNEL_GEMM_F16X3_128;
            ids[1] = MPOW_KERNEL_GEMM_F16X3_256;
            return 2;
        case MPOW_BF16X3:
            ids[0] = MPOW_KERNEL_GEMM_BF16X3_128;
            ids[1] = MPOW_KERNEL_GEMM_BF16X3_256;
            return 2;
        default:
            ids[0] = MPOW_KERNEL_GEMM_BF16X6_128;
            ids[1] = MPOW_KERNEL_GEMM_BF16X6_256;
            return 2;
    }
}
// float32 picks start at n = 768 (below it the whole-K tile with a K split,
// another accumulation order, stays the choice)
int pick_first_bucket(int mode) { return mode == MPOW_FP32 ? 3 : 1; }
int pick_last_bucket(const mpow_plan *plan) {
    const int m = plan->max_n < kPickMaxN ? plan->max_n : kPickMaxN;
    return m / 256;
}

// Cache format (text): a line "mpow-tune <key>", then one line per batch
// size bucket "<n> <shape>" and one per product-pick bucket
// "pick <n> <kernel id>".  A cache serves a plan when its key (GPU model and
// mode) matches and it holds every entry the plan tunes.
bool load_cache(const char *path, const std::string &key, mpow_plan *plan) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool ok = false;
    int got[kBuckets], pick[kPickBuckets];
    for (int b = 0; b < kBuckets; ++b) got[b] = -1;
    for (int b = 0; b < kPickBuckets; ++b) pick[b] = -1;
    if (fgets(line, sizeof line, f)) {
        std::string head(line);
        while (!head.empty() && (head.back() == '\n' || head.back() == '\r')) head.pop_back();
        ok = head == "mpow-tune " + key;
    }
    int ids[4];
    const int nc = pick_candidates(plan->mode, ids);
    while (ok && fgets(line, sizeof line, f)) {
        int n = 0, v = -1;
        if (sscanf(line, "pick %d %d", &n, &v) == 2) {
            bool known = false;
            for (int c = 0; c < nc; ++c) known = known || ids[c] == v;
            if (n % 256 || n < 256 || n > kPickMaxN || !known) {
                ok = false;
                break;
            }
            pick[n / 256] = v;
        } else if (sscanf(line, "%d %d", &n, &v) == 2 && n % 16 == 0 && n >= 16 && n <= kBatchMaxN &&
                   v >= 0 && v < kShapes) {
            got[n / 16] = v;
        } else {
            ok = false;
            break;
        }
    }
    fclose(f);
    if (!ok) return false;
    const bool batch = plan->max_batch > 0 && plan->mode == MPOW_FP32;
    const int bmax = plan->max_n < kBatchMaxN ? plan->max_n : kBatchMaxN;
    if (batch)
        for (int b = 1; b * 16 <= bmax; ++b)
            if (got[b] < 0) return false;
    for (int b = pick_first_bucket(plan->mode); b <= pick_last_bucket(plan); ++b)
        if (pick[b] < 0) return false;
    if (batch)
        for (int b = 1; b * 16 <= bmax; ++b) plan->batch.cfg[b] = got[b];
    for (int b = pick_first_bucket(plan->mode); b <= pick_last_bucket(plan); ++b)
        plan->ws.pick1[b] = (int8_t)(pick[b] + 1);
    return true;
}

bool save_cache(const char *path, const std::string &key, const mpow_plan *plan) {
    FILE *f = fopen(path, "w");
    if (!f) return false;
    fprintf(f, "mpow-tune %s\n", key.c_str());
    if (plan->max_batch > 0 && plan->mode == MPOW_FP32) {
        const int bmax = plan->max_n < kBatchMaxN ? plan->max_n : kBatchMaxN;
        for (int b = 1; b * 16 <= bmax; ++b) fprintf(f, "%d %d\n", b * 16, plan->batch.cfg[b]);
    }
    for (int b = pick_first_bucket(plan->mode); b <= pick_last_bucket(plan); ++b)
        if (plan->ws.pick1[b] > 0) fprintf(f, "pick %d %d\n", 256 * b, plan->ws.pick1[b] - 1);
    return fclose(f) == 0;
}

struct Timer {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool init() {
        return hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    }
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
    // One timed run of fn(s) in ms; < 0 on error.
    template <typename Fn>
    float once_ms(Fn fn) {
        float ms = 0.f;
        if (hipEventRecord(e0, s) != hipSuccess || fn(s) != hipSuccess ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return -1.f;
        return ms;
    }
    // Runs fn(s) for at least `seconds` of device time (and at least once):
    // the clock of a GPU that was idle runs low for its first few hundred
    // milliseconds of work, which would favour the candidates timed last.
    template <typename Fn>
    bool warm(float seconds, Fn fn) {
        float total = 0.f;
        do {
            const float ms = once_ms(fn);
            if (ms < 0.f) return false;
            total += ms;
        } while (total < 1e3f * seconds);
        return true;
    }
    // Index of the fastest of nc candidates: select(c) makes candidate c
    // current, fn(s) runs it; every round times each candidate once, in
    // turn (one untimed round first), and a candidate's time is its fastest.
    // -1 on error.
    template <typename Select, typename Fn>
    int fastest(int nc, int rounds, Select select, Fn fn, float *best_ms = nullptr) {
        float t[8];
        for (int c = 0; c < nc; ++c) t[c] = 1e30f;
        for (int r = 0; r <= rounds; ++r)
            for (int c = 0; c < nc; ++c) {
                select(c);
                const float ms = once_ms(fn);
                if (ms < 0.f) return -1;
                if (r > 0 && ms < t[c]) t[c] = ms;
            }
        int b = 0;
        for (int c = 1; c < nc; ++c)
            if (t[c] < t[b]) b = c;
        if (best_ms) *best_ms = t[b];
        return b;
    }
};

// Any well-scaled dense matrix serves: fixed pseudo-random entries.
void fill_host(std::vector<float> &h, uint32_t &x) {
    for (size_t i = 0; i < h.size(); ++i) {
        x = x * 1664525u + 1013904223u;
        h[i] = ((float)(x >> 8) / 16777216.0f - 0.5f) * 0.2f;
    }
}

mpow_status tune_batch(mpow_plan *plan, Timer &tm) {
    if (batch_wait_all(&plan->batch) != hipSuccess) return MPOW_ERR_DEVICE;
    const int bmax = plan->max_n < kBatchMaxN ? plan->max_n : kBatchMaxN;
    int wmax = 0;
    for (int w : plan->batch.workers) wmax = w > wmax ? w : wmax;
    const int count = plan->max_batch < 2 * wmax ? plan->max_batch : 2 * wmax;
    const size_t mat = (size_t)bmax * bmax;
    float *in = nullptr, *out = nullptr;
    if (hipMalloc((void **)&in, mat * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&out, (size_t)count * mat * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (in) (void)hipFree(in);
        return MPOW_ERR_NOMEM;
    }
    mpow_status st = MPOW_SUCCESS;
    std::vector<float> host(mat);
    uint32_t x = 12345u;
    fill_host(host, x);
    if (hipMemcpy(in, host.data(), mat * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        st = MPOW_ERR_DEVICE;

    int before[kBuckets];
    for (int b = 0; b < kBuckets; ++b) before[b] = plan->batch.cfg[b];
    // Each bucket is timed on a uniform batch of its size through the same
    // grouping and launches as a real batch, once per tile shape.
    std::vector<const float *> Ap((size_t)count, in);
    std::vector<float *> Op((size_t)count);
    std::vector<int> nv((size_t)count);
    std::vector<int64_t> pv((size_t)count, kTuneP);
    for (int i = 0; i < count; ++i) Op[i] = out + (size_t)i * mat;
    auto batch = [&](hipStream_t s) {
        return batch_enqueue(&plan->batch, count, Ap.data(), nv.data(), pv.data(), Op.data(), nullptr,
                             s, false, nullptr);
    };
    for (int i = 0; i < count; ++i) nv[i] = bmax;
    if (st == MPOW_SUCCESS && !tm.warm(0.4f, batch)) st = MPOW_ERR_DEVICE;
    for (int b = 1; st == MPOW_SUCCESS && b * 16 <= bmax; ++b) {
        for (int i = 0; i < count; ++i) nv[i] = b * 16;
        const int prev = plan->batch.cfg[b];
        const int best_shape = tm.fastest(kShapes, 3, [&](int c) { plan->batch.cfg[b] = c; }, batch);
        if (best_shape < 0) st = MPOW_ERR_DEVICE;
        plan->batch.cfg[b] = st == MPOW_SUCCESS ? best_shape : prev;
    }

    // Per-bucket winners on uniform batches can split a mixed batch into
    // several launches that run one after another, each ending in a tail of
    // idle CUs.  So whole tables are also timed on a ragged batch (sizes
    // uniform over the buckets, powers log-uniform in [2, 1000], fixed
    // pseudo-random draws), and the fastest table is kept: the per-bucket
    // one, the table before tuning, and one shape for every size.
    if (st == MPOW_SUCCESS) {
        const int nbk = bmax / 16;
        for (int i = 0; i < count; ++i) {
            x = x * 1664525u + 1013904223u;
            nv[i] = 16 * (1 + (int)((x >> 8) % (uint32_t)nbk));
            x = x * 1664525u + 1013904223u;
            const double u = (double)(x >> 8) / 16777216.0;
            pv[i] = (int64_t)(2.0 * std::exp(u * std::log(500.0)) + 0.5);
        }
        int tables[2 + kShapes][kBuckets];
        for (int b = 0; b < kBuckets; ++b) tables[0][b] = plan->batch.cfg[b];
        for (int b = 0; b < kBuckets; ++b) tables[1][b] = before[b];
        int ntab = 2;
        for (int shape = 0; shape < kShapes; ++shape, ++ntab)
            for (int b = 0; b < kBuckets; ++b) tables[ntab][b] = b == 0 ? before[0] : shape;
        int best_t = tm.fastest(
            ntab, 2, [&](int t) { for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = tables[t][b]; },
            batch);
        if (best_t < 0) {
            st = MPOW_ERR_DEVICE;
            best_t = 1;
        }
        for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = tables[best_t][b];
    }
    if (st == MPOW_SUCCESS && batch_wait_all(&plan->batch) != hipSuccess) st = MPOW_ERR_DEVICE;
    (void)hipFree(in);
    (void)hipFree(out);
    return st;
}

// The single-matrix product kernel per 256-wide size bucket: for n = 256 b
// (every bucket from the mode's first up to min(max_n, 8192)), one power A^2
// (the input's norm, one product, the final rescale; for the split modes
// also the split of A) per candidate on the plan's own workspace, the
// fastest kept.
mpow_status tune_picks(mpow_plan *plan, Timer &tm) {
    const int last = pick_last_bucket(plan);
    const int first = pick_first_bucket(plan->mode);
    if (last < first) return MPOW_SUCCESS;
    const int nmax = 256 * last;
    const size_t mat = (size_t)nmax * nmax;
    float *in = nullptr, *out = nullptr;
    if (hipMalloc((void **)&in, mat * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&out, mat * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (in) (void)hipFree(in);
        return MPOW_ERR_NOMEM;
    }
    mpow_status st = MPOW_SUCCESS;
    std::vector<float> host(mat);
    uint32_t x = 54321u;
    fill_host(host, x);
    if (hipMemcpy(in, host.data(), mat * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        st = MPOW_ERR_DEVICE;
    int ids[4];
    const int nc = pick_candidates(plan->mode, ids);
    Workspace ws = plan->ws;  // the plan's buffers with each candidate forced
    int n = 256 * last;
    auto power = [&](hipStream_t s) { return enqueue_power(ws, in, n, 2, out, nullptr, s, nullptr); };
    ws.kernel = ids[0];
    if (st == MPOW_SUCCESS && !tm.warm(0.3f, power)) st = MPOW_ERR_DEVICE;
    for (int b = first; st == MPOW_SUCCESS && b <= last; ++b) {
        n = 256 * b;
        const int c = tm.fastest(nc, 2, [&](int k) { ws.kernel = ids[k]; }, power);
        if (c < 0) st = MPOW_ERR_DEVICE;
        else plan->ws.pick1[b] = (int8_t)(ids[c] + 1);
    }
    (void)hipFree(in);
    (void)hipFree(out);
    return st;
}

}  // namespace

extern "C" {

mpow_status mpow_plan_tile_table(mpow_plan_t plan, int *table, int len, int set) {
    if (!plan || !table || len < kBuckets || plan->max_batch < 1) return MPOW_ERR_INVALID;
    if (set) {
        for (int b = 0; b < kBuckets; ++b)
            if (table[b] < 0 || table[b] >= kShapes) return MPOW_ERR_INVALID;
        for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = table[b];
    } else {
        for (int b = 0; b < kBuckets; ++b) table[b] = plan->batch.cfg[b];
    }
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_autotune(mpow_plan_t plan, const char *cache_path, uint32_t flags) {
    if (!plan || (flags & ~MPOW_TUNE_FORCE) != 0) return MPOW_ERR_INVALID;
    DevGuard guard(plan->device);
    if (!guard.ok) return MPOW_ERR_DEVICE;
    const std::string key = device_key(plan->device, plan->mode);
    if (cache_path && !(flags & MPOW_TUNE_FORCE) && load_cache(cache_path, key, plan))
        return MPOW_SUCCESS;
    Timer tm;
    mpow_status st = tm.init() ? MPOW_SUCCESS : MPOW_ERR_DEVICE;
    if (st == MPOW_SUCCESS && plan->max_batch > 0 && plan->mode == MPOW_FP32) st = tune_batch(plan, tm);
    if (st == MPOW_SUCCESS) st = tune_picks(plan, tm);
    if (st != MPOW_SUCCESS) plan->last_error = (int)hipGetLastError();
    if (st == MPOW_SUCCESS && cache_path) (void)save_cache(cache_path, key, plan);
    return st;
}

int mpow_plan_kernel_for(mpow_plan_t plan, int n, int aligned) {
    if (!plan || n < 1 || n > plan->max_n) return -1;
    const bool vec4 = aligned != 0 && n % 4 == 0;
    if (plan->mode == MPOW_FP32) {
        const bool window = plan->ws.escaleY != nullptr;
        if (!window && n <= kPowerWgMaxN &&
            (plan->ws.kernel == MPOW_KERNEL_POWER_WG || (plan->ws.kernel < 0 && n <= kPowerWgAutoMaxN)))
            return MPOW_KERNEL_POWER_WG;
        return gemm_resolve(ws_product_kernel(plan->ws, n, vec4), n, vec4);
    }
    return ws_product_kernel(plan->ws, n, vec4);
}

}  // extern "C"
