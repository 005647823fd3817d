// Single-matrix form of the whole-power workgroup (power_wg.h): for small n
// the whole power A^p runs in one launch of one 8-wave workgroup whose base
// and running matrix stay in LDS, instead of one launch per product.
#include "mpow_internal.h"
#include "power_wg.h"

namespace mpow {

namespace {

__global__ __launch_bounds__(512, 1) void power_wg_kernel(const float *A, int n, int64_t p,
                                                          float *out, double *log2_scale) {
    __shared__ __attribute__((aligned(16))) float LX[WgResLds<WG_RES_MAX_N>::FLOATS];
    __shared__ __attribute__((aligned(16))) float LA[WgResLds<WG_RES_MAX_N>::FLOATS];
    __shared__ double red[8];
    wg_power_resident<WG_RES_MAX_N, 8>(A, n, p, out, log2_scale, LX, LA, red);
}

}  // namespace

hipError_t launch_power_wg(const float *A, int n, int64_t p, float *out, double *log2_scale,
                           hipStream_t s) {
    if (n < 1 || n > WG_RES_MAX_N || p < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(power_wg_kernel, dim3(1), dim3(512), 0, s, A, n, p, out, log2_scale);
    return hipGetLastError();
}

}  // namespace mpow
