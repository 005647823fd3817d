// Ragged batch of independent powers in one persistent launch.
//
// Each workgroup is a worker: it claims the next matrix from a queue (an
// atomic counter over descriptors the host sorted by estimated work, largest
// first), computes that matrix's whole power by itself, and claims again
// until the queue is empty.  Every product is the same float32 tile product
// as the single-matrix path (f32_tile), looped over the output tiles of the
// matrix, so each output element is accumulated in exactly the same order as
// in mpow_run's kernels without a K split; the running matrices live in two
// per-worker scratch buffers.  Because one workgroup owns a whole matrix, the
// per-step Frobenius norm is a workgroup reduction and needs no extra launch.
//
// Tile shapes 128x128 and 64x64 (2x2 waves each) and 256x256 (2x4 waves),
// one load path that picks 16- or 4-byte loads at run time, and three
// register-staged kernel instances: every extra tile variant in a kernel
// raises its register allocation (the compiler sizes it for the union of all
// paths), and with eight variants in one kernel it reached one workgroup per
// CU.  Instance 0
// holds only the 64x64 tile (124 registers, four workgroups per CU),
// instance 1 the 128x128 and 64x64 tiles (244 registers, two per CU), and
// instance 2 the 256x256 tile on 8 waves (one per CU).  The host launches the
// smallest instance that holds every tile shape the batch uses.  A fourth
// instance, for batches whose every matrix allows 16-byte loads (n % 4 == 0,
// 16-byte aligned A), runs the 128x128 and 64x64 shapes as the LDS-DMA tiles
// of gemm_f32_dma.h (the same accumulation order, so the same bits wherever
// nothing is subnormal) in place of instance 1.
#include "mpow_internal.h"
#include "gemm_f32_dma.h"
#include "gemm_f32_tile.h"
#include "power_wg.h"

namespace mpow {

namespace {

// Whole-matrix loops of one workgroup keep kUnroll 16-byte loads in flight
// per thread (a loop with one load per iteration waits out the memory
// latency n^2 / 256 times).
constexpr int kUnroll = 8;

template <int NT>
__device__ __forceinline__ double wg_sumsq(const float *__restrict__ M, int n, bool vec, double *red) {
    const int64_t total = (int64_t)n * n;
    double acc = 0.0;
    if (vec) {
        const f4 *M4 = (const f4 *)M;
        const int64_t t4 = total / 4;  // total is a multiple of 16 when n % 4 == 0
        for (int64_t b = threadIdx.x; b < t4; b += NT * kUnroll) {
            f4 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                v[u] = i < t4 ? M4[i] : f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc += (double)v[u][c] * (double)v[u][c];
        }
    } else {
        for (int64_t b = threadIdx.x; b < total; b += NT * kUnroll) {
            float v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                v[u] = i < total ? M[i] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) acc += (double)v[u] * (double)v[u];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int s = NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double S = red[0];
    __syncthreads();
    return S;
}

// out = X * 2^-e (exact power-of-two scaling, split in two float factors).
template <int NT>
__device__ __forceinline__ void wg_scale_copy(const float *__restrict__ X, float *__restrict__ out,
                                              int n, bool vec, PowScale f) {
    const int64_t total = (int64_t)n * n;
    if (vec) {
        const f4 *X4 = (const f4 *)X;
        f4 *O4 = (f4 *)out;
        const int64_t t4 = total / 4;
        for (int64_t b = threadIdx.x; b < t4; b += NT * kUnroll) {
            f4 v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                if (i < t4) v[u] = X4[i];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                if (i < t4) O4[i] = v[u] * f.a * f.b;
            }
        }
    } else {
        for (int64_t b = threadIdx.x; b < total; b += NT * kUnroll) {
            float v[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                if (i < total) v[u] = X[i];
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                if (i < total) out[i] = v[u] * f.a * f.b;
            }
        }
    }
}

// out = ldexp(X, s) in float64, rounded to float32 (overflow to inf,
// underflow to zero).
template <int NT>
__device__ __forceinline__ void wg_ldexp_copy(const float *__restrict__ X, float *__restrict__ out,
                                              int n, int s) {
    const int64_t total = (int64_t)n * n;
    for (int64_t b = threadIdx.x; b < total; b += NT * kUnroll) {
        float v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = b + (int64_t)u * NT;
            if (i < total) v[u] = X[i];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = b + (int64_t)u * NT;
            if (i < total) out[i] = (float)ldexp((double)v[u], s);
        }
    }
}

// One product C = (2^-eX X)(2^-eY Y) over all output tiles of an n x n
// matrix; returns its sum of squares (tile sums added in tile order) to all
// threads.
template <int BM, int BN, int WM, int WN, int KS, int VEC = 2>
__device__ __forceinline__ double wg_product(const float *X, int eX, const float *Y, int eY,
                                             float *C, int n, bool vec, float *As, float *Bs,
                                             double *red, double *bcast) {
    const int tn = (n + BN - 1) / BN, tm = (n + BM - 1) / BM;
    const OperandScales sc{pow2_neg(eX), pow2_neg(eY)};
    auto scales = [&]() { return sc; };
    double S = 0.0;
    for (int t = 0; t < tm * tn; ++t) {
        int nn = n, m0 = (t / tn) * BM, n0 = (t % tn) * BN;
        // Opaque to the optimiser: the tile's per-element address and bounds
        // arithmetic is then computed inside this loop instead of being
        // hoisted out of the product loop, where it would hold registers for
        // the whole matrix.
        asm volatile("" : "+s"(nn), "+s"(m0), "+s"(n0), "+s"(X), "+s"(Y), "+s"(C));
        const double ts =
            f32_tile<BM, BN, WM, WN, VEC, KS>(X, Y, scales, C, nn, m0, n0, As, Bs, red, vec);
        S += ts;  // meaningful in thread 0
    }
    if (threadIdx.x == 0) *bcast = S;
    __syncthreads();
    S = *bcast;
    __syncthreads();
    return S;
}

// The same product with the LDS-DMA tile (16-byte loads, n <= 256).
template <int BM, int BN, int WM, int WN, int BK>
__device__ __forceinline__ double wg_product_dma(const float *X, int eX, const float *Y, int eY,
                                                 float *C, int n, float *As0, float *As1,
                                                 float *Bs0, float *Bs1, double *red,
                                                 double *bcast) {
    const int tn = (n + BN - 1) / BN, tm = (n + BM - 1) / BM;
    auto exps = [&]() { return OperandExps{eX, eY}; };
    double S = 0.0;
    for (int t = 0; t < tm * tn; ++t) {
        int nn = n, m0 = (t / tn) * BM, n0 = (t % tn) * BN;
        asm volatile("" : "+s"(nn), "+s"(m0), "+s"(n0), "+s"(X), "+s"(Y), "+s"(C));
        const double ts = f32_tile_dma<BM, BN, WM, WN, BK, false>(X, Y, exps, C, nn, m0, n0, As0,
                                                                  As1, Bs0, Bs1, red);
        S += ts;  // meaningful in thread 0
    }
    if (threadIdx.x == 0) *bcast = S;
    __syncthreads();
    S = *bcast;
    __syncthreads();
    return S;
}

// Tile shape ids: 0 = 128x128, 1 = 64x64 (both give bit-identical
// products), 2 = 256x256 with 8 waves.  Instances: INST 0 holds only 64x64
// (every cfg runs 64x64), INST 1 holds 128x128 and 64x64, INST 2 (512
// threads, one workgroup per CU) holds 256x256 and, for the other cfgs,
// 128x128 on 8 waves.  All add each output's products in the same order.
template <int INST>
struct BatchInst {
    static constexpr int NT = INST == 2 ? 512 : 256;
    static constexpr int TB = INST == 0 ? 64 : (INST == 1 ? 128 : 256);
    static constexpr int KS = INST == 2 ? 2 : 1;  // K split of the small tile in INST 2
    static constexpr int cmax(int a, int b) { return a > b ? a : b; }
    static constexpr int A_FLOATS =
        INST == 2 ? cmax(F32TileLds<256, 256>::A_FLOATS, F32TileLds<128, 128>::A_FLOATS)
                  : F32TileLds<TB, TB>::A_FLOATS;
    static constexpr int B_FLOATS =
        INST == 2 ? cmax(F32TileLds<256, 256>::B_FLOATS, F32TileLds<128, 128>::B_FLOATS)
                  : F32TileLds<TB, TB>::B_FLOATS;
};

// Next matrix of the launch's group (descriptors begin[g] .. end[g] - 1),
// claimed by thread 0 and broadcast; -1 once the group's queue is empty.
// Contains barriers.
__device__ __forceinline__ int claim_item(BatchHeader *hdr, int g, int *claimed) {
    if (threadIdx.x == 0) *claimed = hdr->begin[g] + atomicAdd(&hdr->counter[g], 1);
    __syncthreads();
    const int it = *claimed;
    __syncthreads();
    return it < hdr->end[g] ? it : -1;
}

// The worker loop: claim matrices until the queue is empty and compute each
// one's whole power; product(cfg, X, eX, Y, eY, C, n, vec) computes one
// product in the workgroup and returns its sum of squares.
template <int NT, typename ProductFn>
__device__ __forceinline__ void run_jobs(const BatchLaunch &b, double *red, int *claimed,
                                         ProductFn product) {
    BatchHeader *hdr = (BatchHeader *)b.desc;
    const BatchItem *items = (const BatchItem *)(hdr + 1);
    float *S0 = b.scratch + (int64_t)blockIdx.x * 2 * b.slot_floats;
    float *S1 = S0 + b.slot_floats;

    for (;;) {
        const int it = claim_item(hdr, b.group, claimed);
        if (it < 0) break;

        const BatchItem item = items[it];
        const int n = item.n;
        const int64_t p = item.p;
        const int64_t total = (int64_t)n * n;

        if (p == 0) {
            for (int64_t i = threadIdx.x; i < total; i += NT) {
                const int64_t r = i / n, c = i - r * n;
                item.out[i] = (r == c) ? 1.0f : 0.0f;
            }
            if (item.scale && threadIdx.x == 0) *item.scale = 0.0;
            __syncthreads();
            continue;
        }

        const bool vec = (n % 4 == 0) && (((uintptr_t)item.A & 15) == 0);
        const double SA = wg_sumsq<NT>(item.A, n, vec, red);
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
                    SX = product(item.cfg, X, eX, Y, eY, C, n, vec);
                    s = mul ? s + (double)eX + (double)eA : 2.0 * (s + (double)eX);
                    X = C;
                    eX = exponent_of_sumsq(SX);
                    ++k;
                }
            }
        }

        // finish: the same arithmetic as the single-matrix finish step
        if (item.scale) {
            const bool vec_out = (n % 4 == 0) && ((((uintptr_t)item.out | (uintptr_t)X) & 15) == 0);
            wg_scale_copy<NT>(X, item.out, n, vec_out, pow2_neg(eX));
            if (threadIdx.x == 0) *item.scale = (SX == 0.0) ? 0.0 : s + (double)eX;
        } else {
            double sc = s;
            sc = sc > 4000.0 ? 4000.0 : (sc < -4000.0 ? -4000.0 : sc);
            wg_ldexp_copy<NT>(X, item.out, n, (int)sc);
        }
        __syncthreads();
    }
}

template <int INST>
__global__ __launch_bounds__(BatchInst<INST>::NT) void batched_kernel(BatchLaunch b) {
    typedef BatchInst<INST> I;
    constexpr int NT = I::NT;
    __shared__ __attribute__((aligned(16))) float As[I::A_FLOATS];
    __shared__ __attribute__((aligned(16))) float Bs[I::B_FLOATS];
    __shared__ double red[NT];
    __shared__ double bcast;
    __shared__ int claimed;
    auto product = [&](int cfg, const float *X, int eX, const float *Y, int eY, float *C, int n,
                       bool vec) -> double {
        if (INST == 2) {
            if (cfg == 2)
                return wg_product<256, 256, 2, 4, 1>(X, eX, Y, eY, C, n, vec, As, Bs, red, &bcast);
            return wg_product<128, 128, 2, 4, 1>(X, eX, Y, eY, C, n, vec, As, Bs, red, &bcast);
        }
        if (INST == 1 && cfg == 0)
            return wg_product<128, 128, 2, 2, 1>(X, eX, Y, eY, C, n, vec, As, Bs, red, &bcast);
        return wg_product<64, 64, 2, 2, 1>(X, eX, Y, eY, C, n, vec, As, Bs, red, &bcast);
    };
    run_jobs<NT>(b, red, &claimed, product);
}

// Instance 3: shapes 0 (128x128, K tile 32) and 1 (64x64, K tile 64) as
// LDS-DMA tiles; every matrix of the batch must allow 16-byte loads.
constexpr int kDmaInstFloats = 4096;  // per LDS buffer: 128 x 32 = 32 x 128 = 64 x 64
__global__ __launch_bounds__(256) void batched_dma_kernel(BatchLaunch b) {
    __shared__ __attribute__((aligned(16))) float As0[kDmaInstFloats];
    __shared__ __attribute__((aligned(16))) float As1[kDmaInstFloats];
    __shared__ __attribute__((aligned(16))) float Bs0[kDmaInstFloats];
    __shared__ __attribute__((aligned(16))) float Bs1[kDmaInstFloats];
    __shared__ double red[256];
    __shared__ double bcast;
    __shared__ int claimed;
    auto product = [&](int cfg, const float *X, int eX, const float *Y, int eY, float *C, int n,
                       bool) -> double {
        if (cfg == 0)
            return wg_product_dma<128, 128, 2, 2, 32>(X, eX, Y, eY, C, n, As0, As1, Bs0, Bs1, red,
                                                      &bcast);
        return wg_product_dma<64, 64, 2, 2, 64>(X, eX, Y, eY, C, n, As0, As1, Bs0, Bs1, red,
                                                &bcast);
    };
    run_jobs<256>(b, red, &claimed, product);
}

// Instances 4-7: every matrix's whole power in one workgroup (power_wg.h).
// 4: resident, row stride 64, four waves (n <= 64; 32 KB of LDS, several
// workgroups per CU); 5: resident, row stride 128, eight waves (n <= 128;
// 128 KB, one per CU); 6: K panels streamed from the worker's scratch
// (2 npad^2 floats), eight waves (n <= 256; 128 KB, one per CU); 7: the
// panel form for n <= 128 (64 KB, two per CU).
// Workgroups per CU the resident instances are compiled for: four of the
// 32 KB form (n <= 64), one of the 128 KB form.
template <int LD>
struct ResPerCu {
    static constexpr int value = LD == 64 ? 4 : 1;
};

template <int LD, int NW>
__global__ __launch_bounds__(NW * 64, ResPerCu<LD>::value) void batched_wg_res_kernel(BatchLaunch b) {
    __shared__ __attribute__((aligned(16))) float LX[WgResLds<LD>::FLOATS];
    __shared__ __attribute__((aligned(16))) float LA[WgResLds<LD>::FLOATS];
    __shared__ double red[NW];
    __shared__ int claimed;
    BatchHeader *hdr = (BatchHeader *)b.desc;
    const BatchItem *items = (const BatchItem *)(hdr + 1);
    for (;;) {
        const int it = claim_item(hdr, b.group, &claimed);
        if (it < 0) break;
        const BatchItem item = items[it];
        wg_power_resident<LD, NW>(item.A, item.n, item.p, item.out, item.scale, LX, LA, red);
    }
}

// Waves of the panel instances: sixteen for n <= 256 (four blocks each),
// eight for n <= 128 (two workgroups per CU).
template <int NPMAX>
struct PanelWaves {
    static constexpr int NW = NPMAX == 256 ? 16 : 8;
};

template <int NPMAX>
__global__ __launch_bounds__(PanelWaves<NPMAX>::NW * 64) void batched_wg_panel_kernel(BatchLaunch b) {
    constexpr int NW = PanelWaves<NPMAX>::NW;
    __shared__ __attribute__((aligned(16))) float L0[WgPanelLds<NPMAX>::STAGE];
    __shared__ __attribute__((aligned(16))) float L1[WgPanelLds<NPMAX>::STAGE];
    __shared__ double red[NW];
    __shared__ int claimed;
    BatchHeader *hdr = (BatchHeader *)b.desc;
    const BatchItem *items = (const BatchItem *)(hdr + 1);
    float *scratch = b.scratch + (int64_t)blockIdx.x * 2 * b.slot_floats;
    for (;;) {
        const int it = claim_item(hdr, b.group, &claimed);
        if (it < 0) break;
        const BatchItem item = items[it];
        wg_power_panel<NPMAX, NW>(item.A, item.n, item.p, item.out, item.scale, scratch, L0, L1, red);
    }
}

}  // namespace

// Default tile shape before tuning: the streamed-panel whole-power form for
// every size, which on MI355X beat the tiled shapes at every size of uniform
// batches of 4096 matrices (by 1% at n = 128 up to 73% at n = 160) and on
// ragged batches.
int batched_cfg_for(int) { return 4; }

int batched_occupancy(int inst) {
    int blocks = 0;
    hipError_t e;
    switch (inst) {
        case 7:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_wg_panel_kernel<128>, 512, 0);
            break;
        case 6:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_wg_panel_kernel<256>,
                                                             PanelWaves<256>::NW * 64, 0);
            break;
        case 5:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_wg_res_kernel<128, 8>, 512, 0);
            break;
        case 4:
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_wg_res_kernel<64, 4>, 256, 0);
            break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_dma_kernel, 256, 0); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel<2>, 512, 0); break;
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel<1>, 256, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, batched_kernel<0>, 256, 0); break;
    }
    if (e != hipSuccess) return 1;
    return blocks < 1 ? 1 : blocks;
}

bool batched_uses_scratch(int inst) { return inst != 4 && inst != 5; }

hipError_t launch_batched(const BatchLaunch &b, int grid, int inst, hipStream_t s) {
    switch (inst) {
        case 7: hipLaunchKernelGGL(batched_wg_panel_kernel<128>, dim3(grid), dim3(512), 0, s, b); break;
        case 6:
            hipLaunchKernelGGL(batched_wg_panel_kernel<256>, dim3(grid), dim3(PanelWaves<256>::NW * 64), 0,
                               s, b);
            break;
        case 5: hipLaunchKernelGGL((batched_wg_res_kernel<128, 8>), dim3(grid), dim3(512), 0, s, b); break;
        case 4: hipLaunchKernelGGL((batched_wg_res_kernel<64, 4>), dim3(grid), dim3(256), 0, s, b); break;
        case 3: hipLaunchKernelGGL(batched_dma_kernel, dim3(grid), dim3(256), 0, s, b); break;
        case 2: hipLaunchKernelGGL(batched_kernel<2>, dim3(grid), dim3(512), 0, s, b); break;
        case 1: hipLaunchKernelGGL(batched_kernel<1>, dim3(grid), dim3(256), 0, s, b); break;
        case 0: hipLaunchKernelGGL(batched_kernel<0>, dim3(grid), dim3(256), 0, s, b); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mpow
