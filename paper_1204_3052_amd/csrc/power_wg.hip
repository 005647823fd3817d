// Single-matrix form of the whole-power workgroup (power_wg.h): for small n
// the whole power A^p runs in one launch of one 8-wave workgroup whose base
// and running matrix stay in LDS, instead of one launch per product.
#include "mpow_internal.h"
#include "power_wg.h"

namespace mpow {

namespace {

__global__ __launch_bounds__(WG_NT, 1) void power_wg_kernel(const float *A, int n, int64_t p,
                                                             float *out, double *log2_scale) {
    __shared__ __attribute__((aligned(16))) float L0[WG_STAGE];
    __shared__ __attribute__((aligned(16))) float L1[WG_STAGE];
    __shared__ double red[WG_NT];
    wg_power<true>(A, n, p, out, log2_scale, nullptr, L0, L1, red);
}

}  // namespace

hipError_t launch_power_wg(const float *A, int n, int64_t p, float *out, double *log2_scale,
                           hipStream_t s) {
    if (n < 1 || n > WG_RES_MAX_N || p < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(power_wg_kernel, dim3(1), dim3(WG_NT), 0, s, A, n, p, out, log2_scale);
    return hipGetLastError();
}

}  // namespace mpow
