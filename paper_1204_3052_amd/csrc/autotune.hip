// Autotuner for the ragged-batch kernel: for every size bucket it times each
// tile shape on a synthetic batch that keeps all workers busy, and keeps the
// fastest.  The paper chose its tile size per problem and per amount of local
// memory by hand (section 4.3.7); here the choice is measured on the device.
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

std::string device_key(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + " cus=" + std::to_string(prop.multiProcessorCount);
}

// Cache format (text): a line "mpow-tune <key>" and then one line per bucket
// "<n> <shape>".
bool load_cache(const char *path, const std::string &key, int *table) {
    FILE *f = fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool ok = false;
    int got[kBuckets];
    for (int b = 0; b < kBuckets; ++b) got[b] = -1;
    if (fgets(line, sizeof line, f)) {
        std::string head(line);
        while (!head.empty() && (head.back() == '\n' || head.back() == '\r')) head.pop_back();
        ok = head == "mpow-tune " + key;
    }
    while (ok && fgets(line, sizeof line, f)) {
        int n = 0, shape = -1;
        if (sscanf(line, "%d %d", &n, &shape) != 2 || n % 16 || n < 16 || n > kBatchMaxN ||
            shape < 0 || shape >= kShapes) {
            ok = false;
            break;
        }
        got[n / 16] = shape;
    }
    fclose(f);
    if (!ok) return false;
    for (int b = 1; b < kBuckets; ++b)
        if (got[b] >= 0) table[b] = got[b];
    return true;
}

bool save_cache(const char *path, const std::string &key, const int *table, int bmax) {
    FILE *f = fopen(path, "w");
    if (!f) return false;
    fprintf(f, "mpow-tune %s\n", key.c_str());
    for (int b = 1; b * 16 <= bmax; ++b) fprintf(f, "%d %d\n", b * 16, table[b]);
    return fclose(f) == 0;
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
    if (!plan || plan->max_batch < 1 || (flags & ~MPOW_TUNE_FORCE) != 0) return MPOW_ERR_INVALID;
    if (plan->mode != MPOW_FP32) return MPOW_ERR_UNSUPPORTED;
    DevGuard guard(plan->device);
    if (!guard.ok) return MPOW_ERR_DEVICE;
    const std::string key = device_key(plan->device);
    const int bmax = plan->max_n < kBatchMaxN ? plan->max_n : kBatchMaxN;
    if (cache_path && !(flags & MPOW_TUNE_FORCE)) {
        int table[kBuckets];
        for (int b = 0; b < kBuckets; ++b) table[b] = plan->batch.cfg[b];
        if (load_cache(cache_path, key, table)) {
            for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = table[b];
            return MPOW_SUCCESS;
        }
    }
    hipError_t e;
    e = batch_wait_all(&plan->batch);
    if (e != hipSuccess) {
        plan->last_error = (int)e;
        return MPOW_ERR_DEVICE;
    }

    int wmax = 0;
    for (int w : plan->batch.workers) wmax = w > wmax ? w : wmax;
    const int count = plan->max_batch < 2 * wmax ? plan->max_batch : 2 * wmax;
    const size_t mat = (size_t)bmax * bmax;
    float *in = nullptr, *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    mpow_status st = MPOW_SUCCESS;
    if (hipMalloc((void **)&in, mat * sizeof(float)) != hipSuccess ||
        hipMalloc((void **)&out, (size_t)count * mat * sizeof(float)) != hipSuccess) {
        (void)hipGetLastError();
        if (in) (void)hipFree(in);
        return MPOW_ERR_NOMEM;
    }
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = MPOW_ERR_DEVICE;
    }

    // Any well-scaled dense matrix serves: fixed pseudo-random entries.
    std::vector<float> host(mat);
    uint32_t x = 12345u;
    for (size_t i = 0; i < mat; ++i) {
        x = x * 1664525u + 1013904223u;
        host[i] = ((float)(x >> 8) / 16777216.0f - 0.5f) * 0.2f;
    }
    if (st == MPOW_SUCCESS && hipMemcpy(in, host.data(), mat * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
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
    for (int b = 1; st == MPOW_SUCCESS && b * 16 <= bmax; ++b) {
        const int n = b * 16;
        for (int i = 0; i < count; ++i) nv[i] = n;
        float best = 1e30f;
        const int prev = plan->batch.cfg[b];
        int best_shape = prev;
        for (int shape = 0; shape < kShapes && st == MPOW_SUCCESS; ++shape) {
            plan->batch.cfg[b] = shape;
            float t_min = 1e30f;
            for (int rep = 0; rep < 4 && st == MPOW_SUCCESS; ++rep) {
                float ms = 0.f;
                if (hipEventRecord(e0, s) != hipSuccess ||
                    batch_enqueue(&plan->batch, count, Ap.data(), nv.data(), pv.data(), Op.data(),
                                  nullptr, s, false, nullptr) != hipSuccess ||
                    hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    st = MPOW_ERR_DEVICE;
                    break;
                }
                if (rep > 0 && ms < t_min) t_min = ms;  // first launch is a warm-up
            }
            if (t_min < best) {
                best = t_min;
                best_shape = shape;
            }
        }
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
        int tables[3 + kShapes][kBuckets];
        int ntab = 0;
        for (int b = 0; b < kBuckets; ++b) tables[0][b] = plan->batch.cfg[b];
        for (int b = 0; b < kBuckets; ++b) tables[1][b] = before[b];
        ntab = 2;
        for (int shape = 0; shape < kShapes; ++shape, ++ntab)
            for (int b = 0; b < kBuckets; ++b) tables[ntab][b] = b == 0 ? before[0] : shape;
        float best = 1e30f;
        int best_t = 0;
        for (int t = 0; t < ntab && st == MPOW_SUCCESS; ++t) {
            for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = tables[t][b];
            float t_min = 1e30f;
            for (int rep = 0; rep < 3 && st == MPOW_SUCCESS; ++rep) {
                float ms = 0.f;
                if (hipEventRecord(e0, s) != hipSuccess ||
                    batch_enqueue(&plan->batch, count, Ap.data(), nv.data(), pv.data(), Op.data(),
                                  nullptr, s, false, nullptr) != hipSuccess ||
                    hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    st = MPOW_ERR_DEVICE;
                    break;
                }
                if (rep > 0 && ms < t_min) t_min = ms;
            }
            if (t_min < best) {
                best = t_min;
                best_t = t;
            }
        }
        for (int b = 0; b < kBuckets; ++b) plan->batch.cfg[b] = tables[st == MPOW_SUCCESS ? best_t : 1][b];
    }
    if (st == MPOW_SUCCESS && batch_wait_all(&plan->batch) != hipSuccess) st = MPOW_ERR_DEVICE;
    if (st != MPOW_SUCCESS) plan->last_error = (int)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipFree(in);
    (void)hipFree(out);
    if (st == MPOW_SUCCESS && cache_path) (void)save_cache(cache_path, key, plan->batch.cfg, bmax);
    return st;
}

}  // extern "C"
