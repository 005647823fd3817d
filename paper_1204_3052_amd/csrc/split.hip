// Split-precision products (modes FP16X3 and BF16X3).
//
// Every float32 operand X is written as two 16-bit matrices,
//   X' = X * 2^(k - e)          (e = floor(log2 ||X||_F), k a fixed shift)
//   hi = rn16(X'),  lo = rn16(X' - hi)
// so that X' = hi + lo to about 22 bits (FP16) or 16 bits (BF16).  A product
// then takes three 16-bit MFMA products accumulated in one float32
// accumulator, dropping the lo*lo term:
//   X'Y' ~= hi_X hi_Y + hi_X lo_Y + lo_X hi_Y.
// For FP16 the fixed shift k = 14 puts the largest entry of a normalised
// matrix (||X'||_F < 2^15) inside FP16 range and keeps typical entries, and
// their lo parts, well above FP16's subnormals (an entry of size 2^-12, the
// typical one of a normalised 4096 x 4096 matrix, becomes 4 and its lo part
// about 2^-10).  BF16 has float32's exponent range and needs no shift.  One
// accumulator instead of separate hi*hi and cross-term accumulators halves
// the accumulator registers, which lets two waves share a SIMD.
//
// split_kernel turns a float32 matrix into hi/lo in two layouts: row-major
// (the left operand: a lane reads 8 consecutive k of its row) and transposed
// (the right operand: row j holds column j, so a lane again reads 8
// consecutive k).  Both are zero-padded to ld = n rounded up to 256, so the
// product kernel's loads need no bounds checks.
#include "mpow_internal.h"
#include "scale_device.h"

namespace mpow {

namespace {

template <typename T>
struct SplitTraits;
template <>
struct SplitTraits<_Float16> {
    static constexpr int kShift = 14;
};
template <>
struct SplitTraits<__bf16> {
    static constexpr int kShift = 0;
};

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Vec8;
template <>
struct Vec8<_Float16> {
    typedef h8 type;
};
template <>
struct Vec8<__bf16> {
    typedef b8 type;
};

template <typename T>
__device__ __forceinline__ v16f mfma16(typename Vec8<T>::type a, typename Vec8<T>::type b, v16f c);
template <>
__device__ __forceinline__ v16f mfma16<_Float16>(h8 a, h8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ v16f mfma16<__bf16>(b8 a, b8 b, v16f c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ split

constexpr int STS = 64;  // split tile edge

template <typename T>
__global__ __launch_bounds__(256) void split_kernel(SplitLaunch s) {
    typedef SplitTraits<T> Tr;
    typedef T V4 __attribute__((ext_vector_type(4)));
    __shared__ double red[256];
    __shared__ T th[STS][STS + 8];
    __shared__ T tl[STS][STS + 8];
    const int tid = threadIdx.x;
    const int n = s.n, ld = s.ld;
    const int eX = exponent_of_sumsq(block_sum_partials<256>(s.part, s.nPart, red));
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && s.eSlot) *s.eSlot = eX;
    const PowScale f = pow2_neg(eX - Tr::kShift);
    const int r0 = blockIdx.y * STS, c0 = blockIdx.x * STS;
    const bool vec = (n % 4) == 0 && ((uintptr_t)s.X & 15) == 0;

#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = tid / 16 + 16 * q, c = (tid % 16) * 4;
        const int gr = r0 + r, gc = c0 + c;
        float v[4] = {0.f, 0.f, 0.f, 0.f};
        if (gr < n) {
            if (vec && gc + 3 < n) {
                const f4 x = *(const f4 *)(s.X + (int64_t)gr * n + gc);
                v[0] = x[0]; v[1] = x[1]; v[2] = x[2]; v[3] = x[3];
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (gc + t < n) v[t] = s.X[(int64_t)gr * n + gc + t];
            }
        }
        V4 hv, lv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float x = v[t] * f.a * f.b;
            const T h = (T)x;
            const T l = (T)(x - (float)h);
            hv[t] = h;
            lv[t] = l;
            th[r][c + t] = h;
            tl[r][c + t] = l;
        }
        // four 16-bit values per 8-byte store (ld and gc are multiples of 4)
        *(V4 *)((T *)s.hi + (int64_t)gr * ld + gc) = hv;
        *(V4 *)((T *)s.lo + (int64_t)gr * ld + gc) = lv;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = tid / 16 + 16 * q, r = (tid % 16) * 4;
        V4 hv, lv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            hv[t] = th[r + t][c];
            lv[t] = tl[r + t][c];
        }
        *(V4 *)((T *)s.hiT + (int64_t)(c0 + c) * ld + r0 + r) = hv;
        *(V4 *)((T *)s.loT + (int64_t)(c0 + c) * ld + r0 + r) = lv;
    }
}

// ------------------------------------------------------------------ product

// SBK is the K extent (16-bit elements) of one LDS tile; rows are padded by 8
// elements so that 16-byte LDS reads are conflict-free.
template <typename T, int BM, int BN, int WM, int WN, int SBK>
__global__ __launch_bounds__(WM *WN * 64) void gemm_split_kernel(SplitGemmLaunch g) {
    typedef SplitTraits<T> Tr;
    typedef typename Vec8<T>::type V8;
    constexpr int SLD = SBK + 8;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;

    __shared__ __attribute__((aligned(16))) T Ah[2][BM * SLD];
    __shared__ __attribute__((aligned(16))) T Al[2][BM * SLD];
    __shared__ __attribute__((aligned(16))) T Bh[2][BN * SLD];
    __shared__ __attribute__((aligned(16))) T Bl[2][BN * SLD];
    __shared__ double red[WM * WN];

    const int n = g.n, ld = g.ld;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int grp = lane >> 5, l32 = lane & 31;
    int tm, tn;
    tile_of_block(blockIdx.x, (n + BM - 1) / BM, (n + BN - 1) / BN, &tm, &tn);
    const int m0 = tm * BM;
    const int n0 = tn * BN;

    // 16-byte chunks: a tile row of SBK elements is SBK/8 chunks.
    constexpr int CPR = SBK / 8;
    constexpr int LA = BM * CPR / NT;
    constexpr int LB = BN * CPR / NT;
    static_assert(LA * NT == BM * CPR && LB * NT == BN * CPR, "load split");
    u4 rah[LA], ral[LA], rbh[LB], rbl[LB];
    const T *__restrict__ xh = (const T *)g.xh;
    const T *__restrict__ xl = (const T *)g.xl;
    const T *__restrict__ yh = (const T *)g.yh;
    const T *__restrict__ yl = (const T *)g.yl;

    auto gload = [&](int k0) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int idx = tid + r * NT;
            const int row = idx / CPR, c = (idx % CPR) * 8;
            const int64_t off = (int64_t)(m0 + row) * ld + k0 + c;
            rah[r] = *(const u4 *)(xh + off);
            ral[r] = *(const u4 *)(xl + off);
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int idx = tid + r * NT;
            const int row = idx / CPR, c = (idx % CPR) * 8;
            const int64_t off = (int64_t)(n0 + row) * ld + k0 + c;
            rbh[r] = *(const u4 *)(yh + off);
            rbl[r] = *(const u4 *)(yl + off);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int r = 0; r < LA; ++r) {
            const int idx = tid + r * NT;
            const int row = idx / CPR, c = (idx % CPR) * 8;
            *(u4 *)(&Ah[buf][row * SLD + c]) = rah[r];
            *(u4 *)(&Al[buf][row * SLD + c]) = ral[r];
        }
#pragma unroll
        for (int r = 0; r < LB; ++r) {
            const int idx = tid + r * NT;
            const int row = idx / CPR, c = (idx % CPR) * 8;
            *(u4 *)(&Bh[buf][row * SLD + c]) = rbh[r];
            *(u4 *)(&Bl[buf][row * SLD + c]) = rbl[r];
        }
    };

    v16f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // m0 / n0 rows beyond n read the zero padding (ld is a multiple of 256).
    const int nk = (n + SBK - 1) / SBK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * SBK);
#pragma unroll
        for (int s = 0; s < SBK / 16; ++s) {
            V8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int off = (wm * TM + i * 32 + l32) * SLD + s * 16 + grp * 8;
                ah[i] = *(const V8 *)(&Ah[cur][off]);
                al[i] = *(const V8 *)(&Al[cur][off]);
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int off = (wn * TN + j * 32 + l32) * SLD + s * 16 + grp * 8;
                bh[j] = *(const V8 *)(&Bh[cur][off]);
                bl[j] = *(const V8 *)(&Bl[cur][off]);
            }
            // per accumulator: hi.hi, then hi.lo, then lo.hi (fixed order)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma16<T>(ah[i], bh[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma16<T>(ah[i], bl[j], acc[i][j]);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) acc[i][j] = mfma16<T>(al[i], bh[j], acc[i][j]);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // C = acc * 2^-2k, an exact power of two.
    const float outScale = ldexpf(1.0f, -2 * Tr::kShift);
    double ss = 0.0;
    float *__restrict__ C = g.C;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * TM + i * 32 + 8 * (r >> 2) + 4 * grp + (r & 3);
                const int col = n0 + wn * TN + j * 32 + l32;
                const float v = acc[i][j][r] * outScale;
                if (row < n && col < n) {
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
        g.partC[blockIdx.x] = t;
    }
}

template <typename T, int BM, int BN, int WM, int WN, int SBK>
hipError_t launch_gemm_split(const SplitGemmLaunch &g, hipStream_t s) {
    const int tiles = ((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_split_kernel<T, BM, BN, WM, WN, SBK>), dim3(tiles), dim3(WM * WN * 64),
                       0, s, g);
    return hipGetLastError();
}

}  // namespace

// Padded leading dimension of the split operands: a multiple of the largest
// product tile, so tiles read zeros past n and need no bounds checks.
int split_ld(int n) { return (n + 255) / 256 * 256; }

hipError_t launch_split(int mode, const SplitLaunch &sl, hipStream_t s) {
    const int t = sl.ld / STS;
    if (mode == MPOW_FP16X3)
        hipLaunchKernelGGL(split_kernel<_Float16>, dim3(t, t), dim3(256), 0, s, sl);
    else
        hipLaunchKernelGGL(split_kernel<__bf16>, dim3(t, t), dim3(256), 0, s, sl);
    return hipGetLastError();
}

// 256 x 256 tiles (8 waves, each 128 x 64, K tile 16) from this size up:
// twice the MFMA work per LDS byte of the 128 x 128 tile.  Both accumulate
// every output in the same order (per 16-wide K chunk: hi.hi, hi.lo, lo.hi),
// so the two give bit-identical results.
constexpr int kSplit256From = 2048;

int gemm_split_pick(int mode, int n) {
    const bool big = n >= kSplit256From;
    if (mode == MPOW_FP16X3) return big ? MPOW_KERNEL_GEMM_F16X3_256 : MPOW_KERNEL_GEMM_F16X3_128;
    return big ? MPOW_KERNEL_GEMM_BF16X3_256 : MPOW_KERNEL_GEMM_BF16X3_128;
}

static int split_tile_edge(int kernel) {
    return (kernel == MPOW_KERNEL_GEMM_F16X3_256 || kernel == MPOW_KERNEL_GEMM_BF16X3_256) ? 256 : 128;
}

int gemm_split_tiles(int kernel, int n) {
    const int e = split_tile_edge(kernel);
    const int t = (n + e - 1) / e;
    return t * t;
}

const char *gemm_split_name(int kernel) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F16X3_128: return "gemm_split_kernel<_Float16,128,128,2,2,32>";
        case MPOW_KERNEL_GEMM_BF16X3_128: return "gemm_split_kernel<__bf16,128,128,2,2,32>";
        case MPOW_KERNEL_GEMM_F16X3_256: return "gemm_split_kernel<_Float16,256,256,2,4,16>";
        case MPOW_KERNEL_GEMM_BF16X3_256: return "gemm_split_kernel<__bf16,256,256,2,4,16>";
        default: return nullptr;
    }
}

hipError_t gemm_split_launch(int kernel, const SplitGemmLaunch &g, hipStream_t s) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F16X3_128: return launch_gemm_split<_Float16, 128, 128, 2, 2, 32>(g, s);
        case MPOW_KERNEL_GEMM_BF16X3_128: return launch_gemm_split<__bf16, 128, 128, 2, 2, 32>(g, s);
        case MPOW_KERNEL_GEMM_F16X3_256: return launch_gemm_split<_Float16, 256, 256, 2, 4, 16>(g, s);
        case MPOW_KERNEL_GEMM_BF16X3_256: return launch_gemm_split<__bf16, 256, 256, 2, 4, 16>(g, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mpow
