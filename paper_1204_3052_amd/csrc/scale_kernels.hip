// Memory-bound kernels around the products: the input's sum of squares, the
// identity for p = 0, and the final rescale that turns the last running
// matrix into the caller's output (the only float64 arithmetic on the path).
#include "mpow_internal.h"
#include "steps_device.h"

namespace mpow {

namespace {

constexpr int kNT = 256;

// Partial sums of squares of A (float64), block b covering one contiguous
// chunk of the n*n elements in a fixed order (sumsq_range).
template <bool VEC>
__global__ __launch_bounds__(kNT) void sumsq_kernel(const float *__restrict__ A, int64_t total,
                                                    int64_t chunk, double *__restrict__ part) {
    __shared__ double red[kNT];
    const int64_t begin = (int64_t)blockIdx.x * chunk;
    const int64_t end = begin + chunk < total ? begin + chunk : total;
    const double S = sumsq_range<kNT, VEC>(A, begin, end, red);
    if (threadIdx.x == 0) part[blockIdx.x] = S;
}

__global__ __launch_bounds__(kNT) void identity_kernel(float *__restrict__ out, int n,
                                                       double *__restrict__ log2_scale) {
    const int64_t total = (int64_t)n * n;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kNT) {
        const int64_t r = i / n, c = i - r * n;
        out[i] = (r == c) ? 1.0f : 0.0f;
    }
    if (log2_scale && blockIdx.x == 0 && threadIdx.x == 0) *log2_scale = 0.0;
}

// Final step.  C holds the last product C_G; its true value is C_G * 2^(s_G),
// where s_G follows from the recorded exponents:
//   square   : s_k = 2 (s_{k-1} + e_{k-1})
//   multiply : s_k = s_{k-1} + e_{k-1} + e_0
// (e_k = floor(log2 ||C_k||_F), C_0 = A, s_0 = 0).  The steps are those of
// the binary schedule of p, or naive_steps multiplications when it is >= 0.
// log2_scale == NULL: out = C_G * 2^(s_G) rounded to float32 via float64.
// Otherwise        : out = C_G * 2^(-e_G) and *log2_scale = s_G + e_G, or
//                    0 when C_G is exactly zero.
__global__ __launch_bounds__(kNT) void finish_kernel(const float *C, int n,
                                                     const double *__restrict__ partC, int nPartC,
                                                     const int *__restrict__ escale, int64_t p,
                                                     int naive_steps, float *out,
                                                     double *__restrict__ log2_scale) {
    // C and out may be the same buffer (p = 1 with out == A): every element is
    // read and then written by the same thread.
    __shared__ double red[kNT];
    __shared__ double sh_sG;
    __shared__ int sh_eG;
    __shared__ int sh_zero;
    const double S = sum_partials<kNT>(partC, nPartC, red);
    if (threadIdx.x == 0) {
        double s = 0.0;
        if (naive_steps > 0) {
            // chained products X <- X.A: s_k = s_{k-1} + e_{k-1} + e_0
            const int e0 = escale[0];
            for (int k = 1; k <= naive_steps; ++k) s = s + (double)escale[k - 1] + (double)e0;
        } else if (naive_steps < 0 && p >= 2) {
            const int e0 = escale[0];
            int k = 1;
            const int top = 63 - __clzll((unsigned long long)p);
            for (int bit = top - 1; bit >= 0; --bit) {
                s = 2.0 * (s + (double)escale[k - 1]);
                ++k;
                if ((p >> bit) & 1) {
                    s = s + (double)escale[k - 1] + (double)e0;
                    ++k;
                }
            }
        }
        sh_sG = s;
        sh_eG = exponent_of_sumsq(S);
        sh_zero = (S == 0.0);
        if (log2_scale && blockIdx.x == 0) *log2_scale = sh_zero ? 0.0 : s + (double)sh_eG;
    }
    __syncthreads();
    finish_range(C, out, n, log2_scale != nullptr, sh_eG, sh_sG,
                 (int64_t)blockIdx.x * kNT + threadIdx.x, (int64_t)gridDim.x * kNT);
}

// Final step of a window schedule: product k made slot dst = slot x . slot y
// with operand exponents eX[k], eY[k]; a slot's log2 scale follows
//   s(dst) = s(x) + eX + s(y) + eY,   s(A) = 0
// (the binary recurrences are the special cases x = y and y = A).  C is the
// result slot's matrix and partC its partial sums; otherwise as finish_kernel.
__global__ __launch_bounds__(kNT) void finish_graph_kernel(const float *C, int n,
                                                           const double *__restrict__ partC,
                                                           int nPartC, const int *__restrict__ eX,
                                                           const int *__restrict__ eY,
                                                           GraphOps g, float *out,
                                                           double *__restrict__ log2_scale) {
    __shared__ double red[kNT];
    __shared__ double sh_sG;
    __shared__ int sh_eG;
    const double S = sum_partials<kNT>(partC, nPartC, red);
    if (threadIdx.x == 0) {
        double s[kSlots];
        for (int i = 0; i < kSlots; ++i) s[i] = 0.0;
        for (int k = 0; k < g.count; ++k)
            s[g.op[k][0]] = s[g.op[k][1]] + (double)eX[k] + s[g.op[k][2]] + (double)eY[k];
        sh_sG = s[g.result];
        sh_eG = exponent_of_sumsq(S);
        if (log2_scale && blockIdx.x == 0) *log2_scale = (S == 0.0) ? 0.0 : sh_sG + (double)sh_eG;
    }
    __syncthreads();
    finish_range(C, out, n, log2_scale != nullptr, sh_eG, sh_sG,
                 (int64_t)blockIdx.x * kNT + threadIdx.x, (int64_t)gridDim.x * kNT);
}

int grid_for(int64_t total, int cap) {
    int64_t g = (total + kNT * 4 - 1) / (kNT * 4);
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

int norm_blocks(int n) {
    const int64_t total = (int64_t)n * n;
    int64_t b = (total + 8191) / 8192;
    if (b < 1) b = 1;
    if (b > kMaxNormBlocks) b = kMaxNormBlocks;
    return (int)b;
}

hipError_t launch_sumsq(const float *A, int n, double *part, int blocks, hipStream_t s) {
    const int64_t total = (int64_t)n * n;
    int64_t chunk = (total + blocks - 1) / blocks;
    const bool vec = (((uintptr_t)A) & 15) == 0;
    if (vec) {
        chunk = (chunk + 3) / 4 * 4;  // every chunk starts on a 16-byte boundary
        hipLaunchKernelGGL(sumsq_kernel<true>, dim3(blocks), dim3(kNT), 0, s, A, total, chunk, part);
    } else {
        hipLaunchKernelGGL(sumsq_kernel<false>, dim3(blocks), dim3(kNT), 0, s, A, total, chunk, part);
    }
    return hipGetLastError();
}

hipError_t launch_identity(float *out, int n, double *log2_scale, hipStream_t s) {
    hipLaunchKernelGGL(identity_kernel, dim3(grid_for((int64_t)n * n, 1024)), dim3(kNT), 0, s,
                       out, n, log2_scale);
    return hipGetLastError();
}

hipError_t launch_finish_graph(const float *C, int n, const double *partC, int nPartC,
                              const int *eX, const int *eY, const GraphOps &g, float *out,
                              double *log2_scale, hipStream_t s) {
    hipLaunchKernelGGL(finish_graph_kernel, dim3(grid_for((int64_t)n * n, 2048)), dim3(kNT), 0, s,
                       C, n, partC, nPartC, eX, eY, g, out, log2_scale);
    return hipGetLastError();
}

hipError_t launch_finish(const float *C, int n, const double *partC, int nPartC,
                         const int *escale, int64_t p, float *out, double *log2_scale,
                         hipStream_t s, int naive_steps) {
    hipLaunchKernelGGL(finish_kernel, dim3(grid_for((int64_t)n * n, 2048)), dim3(kNT), 0, s, C, n,
                       partC, nPartC, escale, p, naive_steps, out, log2_scale);
    return hipGetLastError();
}

}  // namespace mpow
