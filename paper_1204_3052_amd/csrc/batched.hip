// Ragged batch of independent powers in one persistent launch.
//
// Each workgroup is a worker: it claims the next matrix from a queue (an
// atomic counter over descriptors the host sorted by estimated work, largest
// first), computes that matrix's whole power by itself, and claims again
// until the queue is empty.  Every product is the same float32 tile product
// as the single-matrix path (f32_tile), looped over the output tiles of the
// matrix, so each output element is accumulated in exactly the same order as
// in mpow_run; the running matrices live in two per-worker scratch buffers
// that stay in L2.  Because one workgroup owns a whole matrix, the per-step
// Frobenius norm is a workgroup reduction and needs no extra launch.
#include "mpow_internal.h"
#include "gemm_f32_tile.h"

namespace mpow {

namespace {

constexpr int kNT = 256;

// Largest LDS footprint among the tile shapes this kernel uses.
constexpr int kLdsA = F32TileLds<128, 128>::A_FLOATS;
constexpr int kLdsB = F32TileLds<128, 128>::B_FLOATS;

__device__ __forceinline__ double wg_sumsq(const float *__restrict__ M, int n, double *red) {
    const int64_t total = (int64_t)n * n;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < total; i += kNT) {
        const double v = (double)M[i];
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int s = kNT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double S = red[0];
    __syncthreads();
    return S;
}

// One product C = (2^-eX X)(2^-eY Y) over all output tiles of an n x n
// matrix; returns its sum of squares (tile sums added in tile order) to all
// threads.
template <int BM, int BN, bool VEC>
__device__ double wg_product(const float *X, int eX, const float *Y, int eY, float *C, int n,
                             float *As, float *Bs, double *red, double *bcast) {
    const int tn = (n + BN - 1) / BN, tm = (n + BM - 1) / BM;
    const OperandScales sc{pow2_neg(eX), pow2_neg(eY)};
    auto scales = [&]() { return sc; };
    double S = 0.0;
    for (int t = 0; t < tm * tn; ++t) {
        const double ts =
            f32_tile<BM, BN, 2, 2, VEC>(X, Y, scales, C, n, (t / tn) * BM, (t % tn) * BN, As, Bs, red);
        S += ts;  // meaningful in thread 0
    }
    if (threadIdx.x == 0) *bcast = S;
    __syncthreads();
    S = *bcast;
    __syncthreads();
    return S;
}

// Tile shape ids: 0 = 128x128, 1 = 64x64, 2 = 128x64, 3 = 64x128 (all with
// 2x2 waves); every shape gives bit-identical products.
__device__ double product_dispatch(int cfg, bool vec, const float *X, int eX, const float *Y,
                                   int eY, float *C, int n, float *As, float *Bs, double *red,
                                   double *bcast) {
    switch (cfg) {
        case 0:
            return vec ? wg_product<128, 128, true>(X, eX, Y, eY, C, n, As, Bs, red, bcast)
                       : wg_product<128, 128, false>(X, eX, Y, eY, C, n, As, Bs, red, bcast);
        case 2:
            return vec ? wg_product<128, 64, true>(X, eX, Y, eY, C, n, As, Bs, red, bcast)
                       : wg_product<128, 64, false>(X, eX, Y, eY, C, n, As, Bs, red, bcast);
        case 3:
            return vec ? wg_product<64, 128, true>(X, eX, Y, eY, C, n, As, Bs, red, bcast)
                       : wg_product<64, 128, false>(X, eX, Y, eY, C, n, As, Bs, red, bcast);
        default:
            return vec ? wg_product<64, 64, true>(X, eX, Y, eY, C, n, As, Bs, red, bcast)
                       : wg_product<64, 64, false>(X, eX, Y, eY, C, n, As, Bs, red, bcast);
    }
}

__global__ __launch_bounds__(kNT) void batched_kernel(BatchLaunch b) {
    __shared__ __attribute__((aligned(16))) float As[kLdsA];
    __shared__ __attribute__((aligned(16))) float Bs[kLdsB];
    __shared__ double red[kNT];
    __shared__ double bcast;
    __shared__ int claimed;

    BatchHeader *hdr = (BatchHeader *)b.desc;
    const BatchItem *items = (const BatchItem *)(hdr + 1);
    const int count = hdr->count;
    float *S0 = b.scratch + (int64_t)blockIdx.x * 2 * b.slot_floats;
    float *S1 = S0 + b.slot_floats;

    for (;;) {
        if (threadIdx.x == 0) claimed = atomicAdd(&hdr->counter, 1);
        __syncthreads();
        const int it = claimed;
        __syncthreads();
        if (it >= count) break;

        const BatchItem item = items[it];
        const int n = item.n;
        const int64_t p = item.p;
        const int64_t total = (int64_t)n * n;

        if (p == 0) {
            for (int64_t i = threadIdx.x; i < total; i += kNT) {
                const int64_t r = i / n, c = i - r * n;
                item.out[i] = (r == c) ? 1.0f : 0.0f;
            }
            if (item.scale && threadIdx.x == 0) *item.scale = 0.0;
            __syncthreads();
            continue;
        }

        const bool vec = (n % 4 == 0) && (((uintptr_t)item.A & 15) == 0);
        const double SA = wg_sumsq(item.A, n, red);
        const int eA = exponent_of_sumsq(SA);
        const float *X = item.A;  // running matrix; its true value is X * 2^s
        int eX = eA;
        double SX = SA;
        double s = 0.0;
        int k = 0;
        if (p >= 2) {
            const int top = 63 - __clzll((unsigned long long)p);
            for (int bit = top - 1; bit >= 0; --bit) {
                for (int pass = 0; pass < 2; ++pass) {
                    const bool mul = pass == 1;
                    if (mul && !((p >> bit) & 1)) break;
                    float *C = (k & 1) ? S1 : S0;
                    const float *Y = mul ? item.A : X;
                    const int eY = mul ? eA : eX;
                    SX = product_dispatch(item.cfg, vec, X, eX, Y, eY, C, n, As, Bs, red, &bcast);
                    s = mul ? s + (double)eX + (double)eA : 2.0 * (s + (double)eX);
                    X = C;
                    eX = exponent_of_sumsq(SX);
                    ++k;
                }
            }
        }

        // finish: the same arithmetic as the single-matrix finish step
        if (item.scale) {
            const PowScale f = pow2_neg(eX);
            for (int64_t i = threadIdx.x; i < total; i += kNT) item.out[i] = X[i] * f.a * f.b;
            if (threadIdx.x == 0) *item.scale = (SX == 0.0) ? 0.0 : s + (double)eX;
        } else {
            double sc = s;
            sc = sc > 4000.0 ? 4000.0 : (sc < -4000.0 ? -4000.0 : sc);
            const int si = (int)sc;
            for (int64_t i = threadIdx.x; i < total; i += kNT)
                item.out[i] = (float)ldexp((double)X[i], si);
        }
        __syncthreads();
    }
}

}  // namespace

// Default tile shape before tuning: the one that pads n least, larger on ties.
int batched_cfg_for(int n) {
    if (n <= 64) return 1;
    const int p128 = (n + 127) / 128 * 128, p64 = (n + 63) / 64 * 64;
    return p128 * p128 <= p64 * p64 ? 0 : 1;
}

int batched_occupancy() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel, kNT, 0) != hipSuccess)
        return 1;
    return blocks < 1 ? 1 : blocks;
}

hipError_t launch_batched(const BatchLaunch &b, int grid, hipStream_t s) {
    hipLaunchKernelGGL(batched_kernel, dim3(grid), dim3(kNT), 0, s, b);
    return hipGetLastError();
}

}  // namespace mpow
