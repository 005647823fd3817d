// Matrix exponential e^A by scaling and squaring, on the power's kernels.
//
//   e^A = (e^B)^(2^j),  B = A * 2^-j  (exact),  ||B||_F < 1/2 for
//   j = max(0, floor(log2 ||A||_F) + 2)  (or the caller's j)
//
// e^B is its Taylor polynomial of degree 8, evaluated by Horner's rule,
//   X_8 = I + B / 8,   X_k = I + (B X_{k+1}) / k  (k = 7, ..., 1),   T = X_1,
// whose remainder is below sum over k > 8 of (1/2)^k / k! (about 6e-9, under
// float32 resolution).  Each step X_k is one float32 product with the
// identity-adding epilogue C = (1/k) (2^-j A) X_{k+1} + I: the factor 2^-j
// is applied to A on load (exact) and 1/k with the identity in one fused
// multiply-add per element.  X_8 needs no product: 1/8 and 2^-j are powers
// of two, so only its diagonal's + 1 rounds.  The j squarings are the power
// T^(2^j) by the float32 power path (per-step Frobenius normalisation, float64
// log2 scale, final rescale), so e^A = M * 2^s as for a power.
#include <climits>

#include "mpow_internal.h"
#include "scale_device.h"

namespace mpow {

namespace {

constexpr int kNT = 256;
constexpr int kTaylorDegree = 8;  // X_8 = I + B / 8 is exact off the diagonal

__global__ __launch_bounds__(kNT) void taylor_start_kernel(const float *__restrict__ A, int n,
                                                           int j, float *__restrict__ out) {
    const PowScale f = pow2_neg(j + 3);  // 2^-j / 8
    const int64_t total = (int64_t)n * n;
    for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kNT) {
        const int64_t r = i / n, c = i - r * n;
        out[i] = A[i] * f.a * f.b + (r == c ? 1.0f : 0.0f);
    }
}

// floor(log2 ||A||_F) from the partial sums, INT_MIN when the norm is zero or
// not finite (no squarings then).
__global__ __launch_bounds__(kNT) void norm_exponent_kernel(const double *__restrict__ part,
                                                            int nPart, int *__restrict__ e) {
    __shared__ double red[kNT];
    const double S = sum_partials<kNT>(part, nPart, red);
    if (threadIdx.x == 0) *e = (S > 0.0 && isfinite(S)) ? exponent_of_sumsq(S) : INT_MIN;
}

}  // namespace

hipError_t enqueue_norm_exponent(const Workspace &ws, const float *A, int n, int *dev_e,
                                 hipStream_t s) {
    const int nb = norm_blocks(n);
    hipError_t e = launch_sumsq(A, n, ws.partA, nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(norm_exponent_kernel, dim3(1), dim3(kNT), 0, s, ws.partA, nb, dev_e);
    return hipGetLastError();
}

int expm_squarings_for(int e) { return e == INT_MIN ? 0 : (e + 2 > 0 ? e + 2 : 0); }

hipError_t enqueue_expm(const Workspace &ws, float *T, const float *A, int n, int j, float *out,
                        double *log2_scale, hipStream_t s, TimingSink *timing) {
    const int64_t total = (int64_t)n * n;
    int grid = (int)((total + kNT * 4 - 1) / (kNT * 4));
    grid = grid < 1 ? 1 : (grid > 2048 ? 2048 : grid);
    hipLaunchKernelGGL(taylor_start_kernel, dim3(grid), dim3(kNT), 0, s, A, n, j, ws.buf[0]);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    const bool vec4 = (n % 4 == 0) && (((uintptr_t)A & 15) == 0);
    int kernel = ws_product_kernel(ws, n, vec4);
    kernel = gemm_resolve(kernel, n, vec4);
    const double flop = 2.0 * (double)n * (double)n * (double)n;
    const float *Y = ws.buf[0];
    for (int k = kTaylorDegree - 1; k >= 1; --k) {
        GemmLaunch g{};
        g.X = A;
        g.partX = nullptr;
        g.eXfix = j;  // B = 2^-j A on load
        g.Y = Y;
        g.partY = nullptr;
        g.eYfix = 0;
        g.C = (k == 1) ? T : ws.buf[(kTaylorDegree - k) & 1];
        g.partC = ws.part[0];
        g.eSlot = nullptr;
        g.n = n;
        g.alpha = 1.0f / (float)k;
        TimingRecord rec{};
        if (timing && (e = timing->start(kernel, flop, s, &rec)) != hipSuccess) return e;
        if ((e = gemm_launch(kernel, g, vec4, s, true)) != hipSuccess) return e;
        if (timing && (e = timing->stop(&rec, s)) != hipSuccess) return e;
        Y = g.C;
    }
    // e^A = T^(2^j)
    return enqueue_power(ws, T, n, (int64_t)1 << j, out, log2_scale, s, timing);
}

}  // namespace mpow
