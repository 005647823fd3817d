// mpow_run_noalloc: the float32 power of mpow_run without a plan and without
// any device allocation.  Its workspace (the two ping-pong running matrices,
// their per-tile partial sums, the input's partial sums and the per-product
// exponents) is carved from one file-scope device array of fixed size, which
// each GPU the library runs on holds from module load until the process ends.
//
// The array's name is a host-side stand-in in host code, not a device
// address: the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress (with that device current) and only that
// address is handed to kernels.  Every call on a GPU shares that GPU's copy;
// nothing in it has to start at zero (each word a call reads was written
// earlier in the same call), so calls clear nothing.
#include <mutex>

#include "mpow_internal.h"

namespace {

using namespace mpow;

constexpr size_t kScratchBytes = fp32_workspace_bytes(MPOW_NOALLOC_MAX_N);

static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current.
hipError_t scratch_on(int dev, char **ptr) {
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_ptr[dev] = p;
    }
    *ptr = (char *)g_ptr[dev];
    return hipSuccess;
}

bool overlap(const void *a, size_t alen, const void *b, size_t blen) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + blen && y < x + alen;
}

}  // namespace

extern "C" mpow_status mpow_run_noalloc(const float *A, int n, int64_t p, float *out,
                                        double *log2_scale, void *stream) {
    if (!A || !out || n < 1 || p < 0) return MPOW_ERR_INVALID;
    if (n > MPOW_NOALLOC_MAX_N || workspace_bytes(n, MPOW_FP32) > kScratchBytes)
        return MPOW_ERR_UNSUPPORTED;
    const size_t bytes = (size_t)n * (size_t)n * sizeof(float);
    if ((const void *)A != (const void *)out && overlap(A, bytes, out, bytes)) return MPOW_ERR_INVALID;
    if (((uintptr_t)A & 3) || ((uintptr_t)out & 3) || ((uintptr_t)log2_scale & 7))
        return MPOW_ERR_INVALID;
    if (log2_scale &&
        (overlap(log2_scale, sizeof(double), A, bytes) || overlap(log2_scale, sizeof(double), out, bytes)))
        return MPOW_ERR_INVALID;
    const hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return MPOW_ERR_DEVICE;
    }
    if (s) {
        // the workspace is the current device's copy: the stream must run there
        hipDevice_t sdev = -1;
        if (hipStreamGetDevice(s, &sdev) != hipSuccess) {
            (void)hipGetLastError();
            return MPOW_ERR_DEVICE;
        }
        if ((int)sdev != dev) return MPOW_ERR_INVALID;
    }
    char *base = nullptr;
    if (scratch_on(dev, &base) != hipSuccess) {
        (void)hipGetLastError();
        return MPOW_ERR_DEVICE;
    }
    // a float32 workspace laid out for this n (the layout of a plan's)
    Workspace ws;
    workspace_carve(base, n, MPOW_FP32, &ws);
    const hipError_t e = enqueue_power(ws, A, n, p, out, log2_scale, s, nullptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return MPOW_ERR_DEVICE;
    }
    return MPOW_SUCCESS;
}
