// Float32 product C = (2^-eX X)(2^-eY Y) for the squaring and multiply steps
// of the power (the paper's section 4.3 method; its tiled kernel of section
// 4.3.7 is the precedent for staging tiles of both operands in on-chip
// memory, with barriers keeping the shared tiles consistent, section 4.3.6).
//
// CDNA4 design:
//  - v_mfma_f32_32x32x2_f32 does the multiply-adds: each 64-lane wave owns a
//    (32*FM) x (32*FN) block of C in FM*FN accumulator tiles of 16 floats/lane.
//  - The K dimension of a 32-wide LDS tile is split between the two lane
//    halves: lanes 0-31 feed k in [0,16) and lanes 32-63 feed k in [16,32), so
//    a lane's A values for four successive MFMAs are contiguous in a row of
//    the A tile and come from one 16-byte LDS read.
//  - Tiles of X (BM x 32) and Y (32 x BN) are loaded from HBM with coalesced
//    16-byte loads, scaled by the exact power of two 2^-e on the way, and
//    stored to one of two LDS buffers while the other one feeds the MFMAs.
//  - The epilogue writes C and the tile's float64 sum of squares (a fixed
//    reduction order), from which the next step derives its scale.
#include "mpow_internal.h"
#include "scale_device.h"

namespace mpow {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BK = 32;       // K extent of one LDS tile
constexpr int KH = BK / 2;   // K values fed by each lane half
constexpr int ALD = BK + 4;  // LDS row stride of the A tile (floats)

template <int BM, int BN, int WM, int WN, bool VEC>
__global__ __launch_bounds__(WM *WN * 64) void gemm_f32_kernel(GemmLaunch g) {
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;
    constexpr int BLD = BN + 4;
    static_assert(FM >= 1 && FN >= 1 && TM % 32 == 0 && TN % 32 == 0, "wave tile");

    __shared__ __attribute__((aligned(16))) float As[2][BM * ALD];
    __shared__ __attribute__((aligned(16))) float Bs[2][BK * BLD];
    __shared__ double red[NT];

    const int n = g.n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, l32 = lane & 31;

    const int tilesN = (n + BN - 1) / BN;
    const int tile = blockIdx.x;
    const int m0 = (tile / tilesN) * BM;
    const int n0 = (tile % tilesN) * BN;

    // Scales of both operands from their partial sums of squares.
    const int eX = exponent_of_sumsq(block_sum_partials<NT>(g.partX, g.nPartX, red));
    int eY = eX;
    if (g.partY != g.partX) eY = exponent_of_sumsq(block_sum_partials<NT>(g.partY, g.nPartY, red));
    if (blockIdx.x == 0 && tid == 0 && g.eSlot) *g.eSlot = eX;
    const PowScale fx = pow2_neg(eX);
    const PowScale fy = pow2_neg(eY);

    const float *__restrict__ X = g.X;
    const float *__restrict__ Y = g.Y;

    // ---- global -> register staging ------------------------------------
    constexpr int AV = VEC ? 4 : 1;                 // floats per load
    constexpr int LA = BM * BK / (AV * NT);         // loads per thread, A tile
    constexpr int LB = BK * BN / (AV * NT);         // loads per thread, B tile
    static_assert(LA * AV * NT == BM * BK && LB * AV * NT == BK * BN, "load split");
    f4 ra[VEC ? LA : 1];
    f4 rb[VEC ? LB : 1];
    float sa[VEC ? 1 : LA];
    float sb[VEC ? 1 : LB];

    auto gload = [&](int k0) {
        if constexpr (VEC) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
                const int gr = m0 + row, gc = k0 + c;
                f4 v = {0.f, 0.f, 0.f, 0.f};
                if (gr < n && gc < n) v = *(const f4 *)(X + (int64_t)gr * n + gc);
                ra[r] = v;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
                const int gr = k0 + row, gc = n0 + c;
                f4 v = {0.f, 0.f, 0.f, 0.f};
                if (gr < n && gc < n) v = *(const f4 *)(Y + (int64_t)gr * n + gc);
                rb[r] = v;
            }
        } else {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / BK, c = idx % BK;
                const int gr = m0 + row, gc = k0 + c;
                sa[r] = (gr < n && gc < n) ? X[(int64_t)gr * n + gc] : 0.f;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / BN, c = idx % BN;
                const int gr = k0 + row, gc = n0 + c;
                sb[r] = (gr < n && gc < n) ? Y[(int64_t)gr * n + gc] : 0.f;
            }
        }
    };

    auto sstore = [&](int buf) {
        if constexpr (VEC) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
                *(f4 *)(&As[buf][row * ALD + c]) = ra[r] * fx.a * fx.b;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
                *(f4 *)(&Bs[buf][row * BLD + c]) = rb[r] * fy.a * fy.b;
            }
        } else {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                As[buf][(idx / BK) * ALD + idx % BK] = sa[r] * fx.a * fx.b;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                Bs[buf][(idx / BN) * BLD + idx % BN] = sb[r] * fy.a * fy.b;
            }
        }
    };

    v16f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int nk = (n + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const float *as = As[cur];
        const float *bs = Bs[cur];
#pragma unroll
        for (int q = 0; q < KH / 4; ++q) {
            f4 a[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[i] = *(const f4 *)(as + (wm * TM + i * 32 + l32) * ALD + h * KH + 4 * q);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                float b[FN];
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[j] = bs[(h * KH + 4 * q + t) * BLD + wn * TN + j * 32 + l32];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i][t], b[j], acc[i][j],
                                                                        0, 0, 0);
            }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // ---- epilogue: store C and the tile's sum of squares ----------------
    // 32x32 accumulator layout: register r of lane l holds row
    // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the 32x32 block.
    double ss = 0.0;
    float *__restrict__ C = g.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * TM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int col = n0 + wn * TN + j * 32 + l32;
                if (row < n && col < n) {
                    const float v = acc[i][j][r];
                    C[(int64_t)row * n + col] = v;
                    ss += (double)v * (double)v;
                }
            }
    ss = wave_sum_lane0(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WM * WN; ++w) t += red[w];
        g.partC[tile] = t;
    }
}

struct Variant {
    int bm, bn, nt;
    const char *name;
};

// index = MPOW_KERNEL_GEMM_F32_* id
constexpr Variant kVariants[3] = {
    {128, 128, 256, "gemm_f32_kernel<128,128,2,2>"},
    {64, 64, 256, "gemm_f32_kernel<64,64,2,2>"},
    {32, 32, 64, "gemm_f32_kernel<32,32,1,1>"},
};

template <int BM, int BN, int WM, int WN>
hipError_t launch_variant(const GemmLaunch &g, bool vec4, hipStream_t s) {
    const int tiles = ((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    if (vec4)
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, true>), dim3(tiles), dim3(WM * WN * 64),
                           0, s, g);
    else
        hipLaunchKernelGGL((gemm_f32_kernel<BM, BN, WM, WN, false>), dim3(tiles),
                           dim3(WM * WN * 64), 0, s, g);
    return hipGetLastError();
}

}  // namespace

int gemm_pick(int n) {
    if (n >= 1024) return MPOW_KERNEL_GEMM_F32_128;
    if (n >= 256) return MPOW_KERNEL_GEMM_F32_64;
    return MPOW_KERNEL_GEMM_F32_32;
}

int gemm_tiles(int kernel, int n) {
    const Variant &v = kVariants[kernel];
    return ((n + v.bm - 1) / v.bm) * ((n + v.bn - 1) / v.bn);
}

const char *gemm_name(int kernel) {
    if (kernel < 0 || kernel >= 3) return nullptr;
    return kVariants[kernel].name;
}

hipError_t gemm_launch(int kernel, const GemmLaunch &g, bool vec4, hipStream_t s) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F32_128: return launch_variant<128, 128, 2, 2>(g, vec4, s);
        case MPOW_KERNEL_GEMM_F32_64: return launch_variant<64, 64, 2, 2>(g, vec4, s);
        case MPOW_KERNEL_GEMM_F32_32: return launch_variant<32, 32, 1, 1>(g, vec4, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mpow
