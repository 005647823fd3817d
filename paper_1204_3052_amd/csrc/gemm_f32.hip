// Float32 product kernels for the squaring and multiply steps of the power
// (the paper's section 4.3 method): one workgroup per output tile, the tile
// computed by f32_tile (gemm_f32_tile.h).  The prologue derives both operand
// scales from the producers' partial sums of squares; the epilogue records
// the tile's sum of squares for the next step.
#include "mpow_internal.h"
#include "gemm_f32_dma.h"
#include "gemm_f32_tile.h"

namespace mpow {

namespace {

// Both operand exponents of a product from their producers' partial sums of
// squares (an operand without partial sums takes the exponent given in the
// launch); block 0 records them for the log2-scale bookkeeping.  `red` is
// LDS scratch of NT doubles; contains barriers.
template <int NT>
__device__ __forceinline__ OperandExps operand_exponents(const GemmLaunch &g, double *red) {
    if (g.normA) {
        // the input's own sum of squares: thread t adds 16-byte chunks t,
        // t + NT, ... in turn, then the waves' trees and the waves in order
        const f4 *M4 = (const f4 *)g.normA;
        const int t4 = g.n * g.n / 4;
        double acc = 0.0;
        constexpr int U = 8;
        for (int b = threadIdx.x; b < t4; b += NT * U) {
            f4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = b + u * NT;
                v[u] = i < t4 ? M4[i] : f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc += (double)v[u][c] * (double)v[u][c];
        }
        acc = wave_sum_lane0(acc);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        double S = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) S += red[w];
        __syncthreads();  // `red` may be written again
        const int e = exponent_of_sumsq(S);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (g.eSlot) *g.eSlot = e;
            if (g.eSlotY) *g.eSlotY = e;
        }
        return OperandExps{e, e};
    }
    const int eX =
        g.partX ? exponent_of_sumsq(sum_partials<NT>(g.partX, g.nPartX, red)) : g.eXfix;
    int eY = eX;
    if (g.eYin)
        eY = *g.eYin;
    else if (!g.partY)
        eY = g.eYfix;
    else if (g.partY != g.partX)
        eY = exponent_of_sumsq(sum_partials<NT>(g.partY, g.nPartY, red));
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (g.eSlot) *g.eSlot = eX;
        if (g.eSlotY) *g.eSlotY = eY;
    }
    return OperandExps{eX, eY};
}

template <int BM, int BN, int WM, int WN, bool VEC, int KS, bool AXPI>
__global__ __launch_bounds__(WM *WN *KS * 64) void gemm_f32_kernel(GemmLaunch g) {
    constexpr int NT = WM * WN * KS * 64;
    __shared__ __attribute__((aligned(16))) float As[F32TileLds<BM, BN, KS>::A_FLOATS];
    __shared__ __attribute__((aligned(16))) float Bs[F32TileLds<BM, BN, KS>::B_FLOATS];
    __shared__ double red[NT];

    const int n = g.n;
    int tm, tn;
    tile_of_block(blockIdx.x, (n + BM - 1) / BM, (n + BN - 1) / BN, &tm, &tn);
    const int m0 = tm * BM;
    const int n0 = tn * BN;

    // Scales of both operands from their partial sums of squares, reduced
    // while the first tile's loads are in flight.
    auto scales = [&]() {
        const OperandExps e = operand_exponents<NT>(g, red);
        return OperandScales{pow2_neg(e.x), pow2_neg(e.y)};
    };
    const double ss = f32_tile<BM, BN, WM, WN, VEC, KS, AXPI>(g.X, g.Y, scales, g.C, n, m0, n0,
                                                              As, Bs, red, VEC, g.alpha);
    if (threadIdx.x == 0) g.partC[blockIdx.x] = ss;
}

// The tiles fed by LDS-DMA loads (gemm_f32_dma.h), for n % 4 == 0, 16-byte
// aligned operands and n <= DMA_MAX_N.
template <int BM, int BN, int WM, int WN, int BK, bool AXPI>
__global__ __launch_bounds__(WM *WN * 64) void gemm_f32_dma_kernel(GemmLaunch g) {
    constexpr int NT = WM * WN * 64;
    __shared__ __attribute__((aligned(16))) float As0[BM * BK];
    __shared__ __attribute__((aligned(16))) float As1[BM * BK];
    __shared__ __attribute__((aligned(16))) float Bs0[BK * BN];
    __shared__ __attribute__((aligned(16))) float Bs1[BK * BN];
    __shared__ double red[NT];

    const int n = g.n;
    int tm, tn;
    tile_of_block<(BM > BN ? 4 : 8)>(blockIdx.x, (n + BM - 1) / BM, (n + BN - 1) / BN, &tm, &tn);
    auto exps = [&]() { return operand_exponents<NT>(g, red); };
    const double ss = f32_tile_dma<BM, BN, WM, WN, BK, AXPI>(g.X, g.Y, exps, g.C, n, tm * BM,
                                                             tn * BN, As0, As1, Bs0, Bs1, red,
                                                             g.alpha);
    if (threadIdx.x == 0) g.partC[blockIdx.x] = ss;
}

// The 32 x 32 tile with a KS-way K split (KS = 4 or 8 waves) and the whole K
// range in LDS (f32_tile_dma_k4), for n <= DMA_K4_MAX_N with 16-byte loads.
template <int KS, bool AXPI>
__global__ __launch_bounds__(KS * 64) void gemm_f32_dma_k4_kernel(GemmLaunch g) {
    static_assert(DMA_K4_STAGES == 4, "one LDS array per stage below");
    __shared__ __attribute__((aligned(16))) float A0[DMA_K4_A_STAGE];
    __shared__ __attribute__((aligned(16))) float A1[DMA_K4_A_STAGE];
    __shared__ __attribute__((aligned(16))) float A2[DMA_K4_A_STAGE];
    __shared__ __attribute__((aligned(16))) float A3[DMA_K4_A_STAGE];
    __shared__ __attribute__((aligned(16))) float B0[DMA_K4_B_STAGE];
    __shared__ __attribute__((aligned(16))) float B1[DMA_K4_B_STAGE];
    __shared__ __attribute__((aligned(16))) float B2[DMA_K4_B_STAGE];
    __shared__ __attribute__((aligned(16))) float B3[DMA_K4_B_STAGE];
    __shared__ double red[KS * 64];

    const int n = g.n;
    int tm, tn;
    tile_of_block(blockIdx.x, (n + 31) / 32, (n + 31) / 32, &tm, &tn);
    float *const As[4] = {A0, A1, A2, A3};
    float *const Bs[4] = {B0, B1, B2, B3};
    auto exps = [&]() { return operand_exponents<KS * 64>(g, red); };
    const double ss =
        f32_tile_dma_k4<KS, AXPI>(g.X, g.Y, exps, g.C, n, tm * 32, tn * 32, As, Bs, g.alpha);
    if (threadIdx.x == 0) g.partC[blockIdx.x] = ss;
}

struct Variant {
    int id, bm, bn, wm, wn, ks;
    const char *name;
};

// The variants without a K split accumulate each output element in the same
// order (K tiles of 32, same k-to-lane mapping), so they give bit-identical
// products; a K-split variant adds its partial sums in its own fixed order.
constexpr Variant kVariants[] = {
    {MPOW_KERNEL_GEMM_F32_128, 128, 128, 2, 2, 1, "gemm_f32_kernel<128,128,2,2>"},
    {MPOW_KERNEL_GEMM_F32_64, 64, 64, 2, 2, 1, "gemm_f32_kernel<64,64,2,2>"},
    {MPOW_KERNEL_GEMM_F32_32, 32, 32, 1, 1, 1, "gemm_f32_kernel<32,32,1,1>"},
    {MPOW_KERNEL_GEMM_F32_256, 256, 256, 2, 4, 1, "gemm_f32_dma_kernel<256,256,2,4>"},
    {MPOW_KERNEL_GEMM_F32_128x64, 128, 64, 2, 2, 1, "gemm_f32_kernel<128,64,2,2>"},
    {MPOW_KERNEL_GEMM_F32_32_K4, 32, 32, 1, 1, 4, "gemm_f32_kernel<32,32,1,1,K4>"},
    {MPOW_KERNEL_GEMM_F32_32_K8, 32, 32, 1, 1, 8, "gemm_f32_kernel<32,32,1,1,K8>"},
    {MPOW_KERNEL_GEMM_F32_64_K2, 64, 64, 2, 2, 2, "gemm_f32_kernel<64,64,2,2,K2>"},
    {MPOW_KERNEL_GEMM_F32_128_K2, 128, 128, 2, 2, 2, "gemm_f32_kernel<128,128,2,2,K2>"},
    {MPOW_KERNEL_GEMM_F32_64_DMA, 64, 64, 2, 2, 1, "gemm_f32_dma_kernel<64,64,2,2>"},
    {MPOW_KERNEL_GEMM_F32_128_DMA, 128, 128, 4, 2, 1, "gemm_f32_dma_kernel<128,128,4,2>"},
    {MPOW_KERNEL_GEMM_F32_256x128_DMA, 256, 128, 4, 2, 1, "gemm_f32_dma_kernel<256,128,4,2>"},
    {MPOW_KERNEL_GEMM_F32_32_K4_DMA, 32, 32, 1, 1, 4, "gemm_f32_dma_k4_kernel<4>"},
    {MPOW_KERNEL_GEMM_F32_32_K8_DMA, 32, 32, 1, 1, 8, "gemm_f32_dma_k4_kernel<8>"},
};

const Variant *variant(int id) {
    for (const Variant &v : kVariants)
        if (v.id == id) return &v;
    return nullptr;
}

template <int BM, int BN, int WM, int WN, int KS = 1>
hipError_t launch_variant(const GemmLaunch &g, bool vec4, bool axpi, hipStream_t s) {
    const int tiles = ((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    const dim3 block(WM * WN * KS * 64);
    if (axpi) {
        if (vec4)
            hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, true, KS, true>), dim3(tiles), block, 0, s, g);
        else
            hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, false, KS, true>), dim3(tiles), block, 0, s, g);
    } else {
        if (vec4)
            hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, true, KS, false>), dim3(tiles), block, 0, s, g);
        else
            hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, false, KS, false>), dim3(tiles), block, 0, s, g);
    }
    return hipGetLastError();
}

}  // namespace

// Default product kernel per size.  Below n = 768 the output tiles alone
// cannot fill 256 CUs, so 32 x 32 tiles with the K range split over several
// waves (more work per output tile): with 16-byte loads and n <= 512 the
// whole-K-in-LDS form with 8 waves (chains of products measured on MI355X
// with each kernel forced: n = 512, p = 1023 in 0.146 ms against 0.153 ms
// with 4 waves and 0.177-0.181 ms for the register-staged forms; n = 384:
// 0.125 against 0.130 ms), otherwise the register-staged tile with 4 waves.
// From n = 768 with 16-byte loads: the LDS-DMA tile whose estimated rate is
// highest, the estimate being the tile's rate when every CU runs whole waves
// of tiles (measured on MI355X products at n = 4096 ... 8192) times the
// fraction of the last wave of workgroups that is filled:
//   rate = R * (T / 256) / ceil(T / 256),   T = tiles of the n x n output.
// Against per-size measurements from n = 768 to 8192 this picks the fastest
// LDS-DMA tile, or one within 2% of it.
int gemm_pick(int n, bool vec4) {
    if (n < 768)
        return (vec4 && n <= DMA_K4_MAX_N) ? MPOW_KERNEL_GEMM_F32_32_K8_DMA
                                           : MPOW_KERNEL_GEMM_F32_32_K4;
    if (vec4 && n <= DMA_MAX_N) {
        struct Cand {
            int id, bm, bn;
            double rate;  // TFLOP/s with whole waves of tiles
        };
        constexpr Cand cands[] = {
            {MPOW_KERNEL_GEMM_F32_256x128_DMA, 256, 128, 151.0},
            {MPOW_KERNEL_GEMM_F32_256, 256, 256, 149.0},
            {MPOW_KERNEL_GEMM_F32_128_DMA, 128, 128, 147.0},
            {MPOW_KERNEL_GEMM_F32_64_DMA, 64, 64, 141.0},
        };
        int best = MPOW_KERNEL_GEMM_F32_64_DMA;
        double best_rate = 0.0;
        for (const Cand &c : cands) {
            const double rate = tile_fill_rate(c.rate, n, c.bm, c.bn);
            if (rate > best_rate) {
                best_rate = rate;
                best = c.id;
            }
        }
        return best;
    }
    if (n >= 4096) return vec4 ? MPOW_KERNEL_GEMM_F32_256 : MPOW_KERNEL_GEMM_F32_128;
    if (n >= 2560) return MPOW_KERNEL_GEMM_F32_64;
    if (n >= 1792) return MPOW_KERNEL_GEMM_F32_128_K2;
    return MPOW_KERNEL_GEMM_F32_64_K2;
}

bool gemm_is_f32(int kernel) { return variant(kernel) != nullptr; }

int gemm_tiles(int kernel, int n) {
    const Variant *v = variant(kernel);
    return ((n + v->bm - 1) / v->bm) * ((n + v->bn - 1) / v->bn);
}

const char *gemm_name(int kernel) {
    const Variant *v = variant(kernel);
    return v ? v->name : nullptr;
}

template <int BM, int BN, int WM, int WN, int BK>
hipError_t launch_dma(const GemmLaunch &g, bool vec4, bool axpi, hipStream_t s) {
    if (!vec4 || g.n > DMA_MAX_N) return hipErrorInvalidValue;  // unresolved id
    const dim3 grid(((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN)), block(WM * WN * 64);
    if (axpi)
        hipLaunchKernelGGL((gemm_f32_dma_kernel<BM, BN, WM, WN, BK, true>), grid, block, 0, s, g);
    else
        hipLaunchKernelGGL((gemm_f32_dma_kernel<BM, BN, WM, WN, BK, false>), grid, block, 0, s, g);
    return hipGetLastError();
}

int gemm_resolve(int kernel, int n, bool vec4) {
    const bool dma = vec4 && n <= DMA_MAX_N;
    switch (kernel) {
        // the whole-power kernel is not a product kernel: where a product
        // kernel is needed, the per-size default runs
        case MPOW_KERNEL_POWER_WG: return gemm_pick(n, vec4);
        case MPOW_KERNEL_GEMM_F32_256: return vec4 ? kernel : MPOW_KERNEL_GEMM_F32_128;
        case MPOW_KERNEL_GEMM_F32_64_DMA: return dma ? kernel : MPOW_KERNEL_GEMM_F32_64;
        case MPOW_KERNEL_GEMM_F32_128_DMA:
        case MPOW_KERNEL_GEMM_F32_256x128_DMA: return dma ? kernel : MPOW_KERNEL_GEMM_F32_128;
        case MPOW_KERNEL_GEMM_F32_32_K4_DMA:
            return vec4 && n <= DMA_K4_MAX_N ? kernel : MPOW_KERNEL_GEMM_F32_32_K4;
        case MPOW_KERNEL_GEMM_F32_32_K8_DMA:
            return vec4 && n <= DMA_K4_MAX_N ? kernel : MPOW_KERNEL_GEMM_F32_32_K8;
        default: return kernel;
    }
}

hipError_t gemm_launch(int kernel, const GemmLaunch &g, bool vec4, hipStream_t s, bool axpi) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F32_128: return launch_variant<128, 128, 2, 2>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_64: return launch_variant<64, 64, 2, 2>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_32: return launch_variant<32, 32, 1, 1>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_256:
            // 16-byte loads only: the 4-byte-load form of this tile would spill
            if (!vec4) return hipErrorInvalidValue;
            if (g.n <= DMA_MAX_N) return launch_dma<256, 256, 2, 4, 32>(g, vec4, axpi, s);
            if (axpi)
                hipLaunchKernelGGL((gemm_f32_kernel<256, 256, 2, 4, true, 1, true>),
                                   dim3(gemm_tiles(kernel, g.n)), dim3(512), 0, s, g);
            else
                hipLaunchKernelGGL((gemm_f32_kernel<256, 256, 2, 4, true, 1, false>),
                                   dim3(gemm_tiles(kernel, g.n)), dim3(512), 0, s, g);
            return hipGetLastError();
        case MPOW_KERNEL_GEMM_F32_64_DMA: return launch_dma<64, 64, 2, 2, 32>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_128_DMA: return launch_dma<128, 128, 4, 2, 32>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_256x128_DMA:
            return launch_dma<256, 128, 4, 2, 32>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_32_K4_DMA: {
            if (!vec4 || g.n > DMA_K4_MAX_N) return hipErrorInvalidValue;  // unresolved id
            const dim3 grid(gemm_tiles(kernel, g.n)), block(256);
            if (axpi)
                hipLaunchKernelGGL((gemm_f32_dma_k4_kernel<4, true>), grid, block, 0, s, g);
            else
                hipLaunchKernelGGL((gemm_f32_dma_k4_kernel<4, false>), grid, block, 0, s, g);
            return hipGetLastError();
        }
        case MPOW_KERNEL_GEMM_F32_32_K8_DMA: {
            if (!vec4 || g.n > DMA_K4_MAX_N) return hipErrorInvalidValue;  // unresolved id
            const dim3 grid(gemm_tiles(kernel, g.n)), block(512);
            if (axpi)
                hipLaunchKernelGGL((gemm_f32_dma_k4_kernel<8, true>), grid, block, 0, s, g);
            else
                hipLaunchKernelGGL((gemm_f32_dma_k4_kernel<8, false>), grid, block, 0, s, g);
            return hipGetLastError();
        }
        case MPOW_KERNEL_GEMM_F32_128x64: return launch_variant<128, 64, 2, 2>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_32_K4: return launch_variant<32, 32, 1, 1, 4>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_32_K8: return launch_variant<32, 32, 1, 1, 8>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_64_K2: return launch_variant<64, 64, 2, 2, 2>(g, vec4, axpi, s);
        case MPOW_KERNEL_GEMM_F32_128_K2: return launch_variant<128, 128, 2, 2, 2>(g, vec4, axpi, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mpow
