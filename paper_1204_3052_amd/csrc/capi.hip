// C ABI for plans: argument checks, the product schedule of p, plan and
// workspace ownership; the enqueueing itself lives in runtime.hip.
#include <new>

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
    (void)hipGetLastError();
    return MPOW_ERR_DEVICE;
}

constexpr int kWorkersForSizing = 1024;  // 256 CUs x 4 resident workers

int batch_bmax(int max_n) { return max_n < kBatchMaxN ? max_n : kBatchMaxN; }

// [a, a + alen) and [b, b + blen) share at least one byte
bool ranges_overlap(const void *a, size_t alen, const void *b, size_t blen) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + blen && y < x + alen;
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
        case MPOW_ERR_TIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

int mpow_gemm_count(int64_t p) {
    if (p < 0) return -1;
    if (p < 2) return 0;
    const int top = 63 - __builtin_clzll((unsigned long long)p);
    return top + __builtin_popcountll((unsigned long long)p) - 1;
}

int mpow_window_schedule(int64_t p, int w, uint8_t *ops, int cap, int *result) {
    if (p < 1 || w < 0 || w > 3 || !result) return -1;
    if (w == 0) {  // the fewest products over w = 1, 2, 3 (smaller w on ties)
        int best = -1, bw = 1;
        for (int v = 1; v <= 3; ++v) {
            int r = 0;
            const int g = window_schedule(p, v, nullptr, 0, &r);
            if (g >= 0 && (best < 0 || g < best)) {
                best = g;
                bw = v;
            }
        }
        w = bw;
    }
    return window_schedule(p, w, ops, cap, result);
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
    if (max_n < 1 || max_batch < 0 || mode < 0 || mode > MPOW_BF16X6) return 0;
    size_t total = workspace_bytes(max_n, mode);
    if (max_batch > 0) total += batch_device_bytes(max_batch, batch_bmax(max_n), kWorkersForSizing);
    return total;
}

mpow_status mpow_plan_create(mpow_plan_t *out_plan, int device, int max_n, int max_batch,
                             int mode, uint32_t flags) {
    if (!out_plan) return MPOW_ERR_INVALID;
    *out_plan = nullptr;
    if (max_n < 1 || max_batch < 0 || mode < 0 || mode > MPOW_BF16X6 ||
        (flags & ~(MPOW_FLAG_TIMING | MPOW_FLAG_POISON | MPOW_FLAG_EXPM | MPOW_FLAG_WINDOW |
                   MPOW_FLAG_SPLIT_PASS)) != 0)
        return MPOW_ERR_INVALID;
    if ((flags & MPOW_FLAG_WINDOW) && mode != MPOW_FP32) return MPOW_ERR_UNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return MPOW_ERR_DEVICE;
    }
    DeviceGuard guard(device);
    if (!guard.ok) return MPOW_ERR_DEVICE;
    int workers[kBatchInstances] = {};
    if (max_batch > 0 && !batch_workers_for(device, workers)) return MPOW_ERR_DEVICE;
    const int wmax = batch_scratch_workers(workers);
    const size_t ws_bytes = workspace_bytes(max_n, mode);
    const size_t b_bytes = max_batch > 0 ? batch_device_bytes(max_batch, batch_bmax(max_n), wmax) : 0;
    // mpow_expm's Taylor polynomial and norm exponent
    const bool expm = (flags & MPOW_FLAG_EXPM) && mode == MPOW_FP32;
    const size_t e_bytes = expm ? round_up((size_t)max_n * max_n * sizeof(float), 256) + 256 : 0;
    // window schedules: A^2, A^3, A^5, A^7, their partial sums, the eY record
    const bool window = (flags & MPOW_FLAG_WINDOW) != 0;
    const size_t t32 = ((size_t)max_n + 31) / 32;
    const size_t wbuf = round_up((size_t)max_n * max_n * sizeof(float), 256);
    const size_t wpart = round_up(t32 * t32 * sizeof(double), 256);
    const size_t w_bytes = window ? 4 * (wbuf + wpart) + round_up(kMaxGraphOps * sizeof(int), 256) : 0;

    mpow_plan *plan = new (std::nothrow) mpow_plan();
    if (!plan) return MPOW_ERR_NOMEM;
    plan->device = device;
    plan->max_n = max_n;
    plan->max_batch = max_batch;
    plan->mode = mode;
    plan->flags = flags;

    if (hipMalloc((void **)&plan->base, ws_bytes + b_bytes + e_bytes + w_bytes) != hipSuccess ||
        !plan->base) {
        (void)hipGetLastError();
        delete plan;
        return MPOW_ERR_NOMEM;
    }
    if (expm) {
        plan->expm_T = (float *)(plan->base + ws_bytes + b_bytes);
        plan->expm_e_dev = (int *)(plan->base + ws_bytes + b_bytes + e_bytes - 256);
        if (hipHostMalloc((void **)&plan->expm_e_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(plan->base);
            delete plan;
            return MPOW_ERR_NOMEM;
        }
    }
    if (hipMemset(plan->base, (flags & MPOW_FLAG_POISON) ? 0xFF : 0,
                  ws_bytes + b_bytes + e_bytes + w_bytes) != hipSuccess) {
        if (plan->expm_e_host) (void)hipHostFree(plan->expm_e_host);
        (void)hipFree(plan->base);
        delete plan;
        return MPOW_ERR_DEVICE;
    }
    workspace_carve(plan->base, max_n, mode, &plan->ws);
    plan->ws.split_pass = (flags & MPOW_FLAG_SPLIT_PASS) != 0;
    if (window) {
        char *q = plan->base + ws_bytes + b_bytes + e_bytes;
        for (int i = 0; i < 4; ++i) {
            plan->ws.wp[i] = (float *)q; q += wbuf;
            plan->ws.wpart[i] = (double *)q; q += wpart;
        }
        plan->ws.escaleY = (int *)q;
    }
    if (max_batch > 0 &&
        batch_context_init(&plan->batch, plan->base + ws_bytes, max_batch, batch_bmax(max_n),
                           workers) != hipSuccess) {
        (void)hipGetLastError();
        batch_context_release(&plan->batch);
        if (plan->expm_e_host) (void)hipHostFree(plan->expm_e_host);
        (void)hipFree(plan->base);
        delete plan;
        return MPOW_ERR_NOMEM;
    }
    *out_plan = plan;
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_destroy(mpow_plan_t plan) {
    if (!plan) return MPOW_SUCCESS;
    DeviceGuard guard(plan->device);
    (void)hipDeviceSynchronize();
    plan->timing.destroy();
    batch_context_release(&plan->batch);
    if (plan->expm_e_host) (void)hipHostFree(plan->expm_e_host);
    (void)hipFree(plan->base);
    delete plan;
    return MPOW_SUCCESS;
}

int mpow_last_device_error(mpow_plan_t plan) { return plan ? plan->last_error : 0; }

namespace {

mpow_status check_run_args(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                           double *log2_scale) {
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
    return MPOW_SUCCESS;
}

}  // namespace

mpow_status mpow_run(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                     double *log2_scale, void *stream) {
    const mpow_status st = check_run_args(plan, A, n, p, out, log2_scale);
    if (st != MPOW_SUCCESS) return st;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    TimingSink *t = (plan->flags & MPOW_FLAG_TIMING) ? &plan->timing : nullptr;
    const hipError_t e = enqueue_power(plan->ws, A, n, p, out, log2_scale, (hipStream_t)stream, t);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

mpow_status mpow_run_naive(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                           double *log2_scale, void *stream) {
    const mpow_status st = check_run_args(plan, A, n, p, out, log2_scale);
    if (st != MPOW_SUCCESS) return st;
    if (p > MPOW_NAIVE_MAX_P) return MPOW_ERR_INVALID;
    if (plan->mode != MPOW_FP32) return MPOW_ERR_UNSUPPORTED;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    TimingSink *t = (plan->flags & MPOW_FLAG_TIMING) ? &plan->timing : nullptr;
    const hipError_t e =
        enqueue_power_naive(plan->ws, A, n, p, out, log2_scale, (hipStream_t)stream, t);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

mpow_status mpow_expm(mpow_plan_t plan, const float *A, int n, float *out, double *log2_scale,
                      int squarings, void *stream) {
    const mpow_status st = check_run_args(plan, A, n, 1, out, log2_scale);
    if (st != MPOW_SUCCESS) return st;
    if (squarings < -1 || squarings > 62) return MPOW_ERR_INVALID;
    if (plan->mode != MPOW_FP32 || !plan->expm_T) return MPOW_ERR_UNSUPPORTED;
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    const hipStream_t s = (hipStream_t)stream;
    int j = squarings;
    if (j < 0) {
        hipError_t e = enqueue_norm_exponent(plan->ws, A, n, plan->expm_e_dev, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(plan->expm_e_host, plan->expm_e_dev, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return device_error(plan, e);
        j = expm_squarings_for(*plan->expm_e_host);
        if (j > 62) return MPOW_ERR_UNSUPPORTED;
    }
    TimingSink *t = (plan->flags & MPOW_FLAG_TIMING) ? &plan->timing : nullptr;
    const hipError_t e = enqueue_expm(plan->ws, plan->expm_T, A, n, j, out, log2_scale, s, t);
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
    DeviceGuard guard(plan->device);
    if (!guard.ok) return device_error(plan, hipErrorInvalidDevice);
    std::vector<double *> scales;
    if (log2_scale) {
        scales.resize(count);
        for (int i = 0; i < count; ++i) scales[i] = log2_scale + i;
    }
    const hipError_t e = batch_enqueue(&plan->batch, count, A, n, p, out,
                                       log2_scale ? scales.data() : nullptr, (hipStream_t)stream,
                                       true);
    return e == hipSuccess ? MPOW_SUCCESS : device_error(plan, e);
}

int mpow_mode_for_tolerance(double tol, double floor, int wide_range) {
    if (!(tol >= 0.0) || !(floor >= 0.0)) return -1;  // also rejects NaN
    // stated bars: max(ABS, FACTOR * floor)
    const double fp32_class = floor * 64.0 > 1e-5 ? floor * 64.0 : 1e-5;
    const double bf16x3 = floor * 1024.0 > 2e-4 ? floor * 1024.0 : 2e-4;
    if (bf16x3 <= tol) return MPOW_BF16X3;
    if (fp32_class <= tol) return wide_range ? MPOW_BF16X6 : MPOW_FP16X3;
    return -1;
}

int mpow_fp32_kernel_for(int n, int aligned) {
    if (n < 1) return -1;
    const bool vec4 = aligned != 0 && n % 4 == 0;
    return gemm_resolve(gemm_pick(n, vec4), n, vec4);
}

mpow_status mpow_plan_set_kernel(mpow_plan_t plan, int kernel) {
    if (!plan) return MPOW_ERR_INVALID;
    bool ok = kernel == -1;
    if (!ok && plan->mode == MPOW_FP32) ok = gemm_is_f32(kernel) || kernel == MPOW_KERNEL_POWER_WG;
    if (!ok && plan->mode != MPOW_FP32) ok = gemm_split_mode(kernel) == plan->mode;
    if (!ok) return MPOW_ERR_INVALID;
    plan->ws.kernel = kernel;
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_timing(mpow_plan_t plan, int kernel, int64_t *launches, double *total_ms,
                             double *total_flop, const char **name) {
    if (!plan || !(plan->flags & MPOW_FLAG_TIMING) || kernel < 0 || kernel >= MPOW_KERNEL_COUNT)
        return MPOW_ERR_INVALID;
    DeviceGuard guard(plan->device);
    const hipError_t e = plan->timing.collect();
    if (e != hipSuccess) return device_error(plan, e);
    if (launches) *launches = plan->timing.launches[kernel];
    if (total_ms) *total_ms = plan->timing.ms[kernel];
    if (total_flop) *total_flop = plan->timing.flop[kernel];
    if (name)
        *name = kernel == MPOW_KERNEL_POWER_WG ? "power_wg_kernel"
                : gemm_name(kernel)            ? gemm_name(kernel)
                                               : gemm_split_name(kernel);
    return MPOW_SUCCESS;
}

mpow_status mpow_plan_timing_reset(mpow_plan_t plan) {
    if (!plan) return MPOW_ERR_INVALID;
    mpow_status st = MPOW_SUCCESS;
    if (plan->flags & MPOW_FLAG_TIMING) {
        DeviceGuard guard(plan->device);
        const hipError_t e = plan->timing.collect();
        if (e != hipSuccess) st = device_error(plan, e);
    }
    plan->timing.reset();
    return st;
}

}  // extern "C"
