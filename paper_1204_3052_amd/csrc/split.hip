// Split-precision products (modes FP16X3, BF16X3 and BF16X6).
//
// Every float32 operand X is written as NP 16-bit matrices,
//   X' = X * 2^(k - e)          (e = floor(log2 ||X||_F), k a fixed shift)
//   x0 = rn16(X'),  x1 = rn16(X' - x0),  x2 = rn16(X' - x0 - x1)
// (each difference is exact in float32), so that X' = x0 + x1 (+ x2) to about
// 22 bits (FP16, NP = 2), 16 bits (BF16, NP = 2) or 24 bits (BF16, NP = 3).
// A product then takes the 16-bit MFMA products x_i y_j with i + j < NP
// (three for NP = 2, six for NP = 3: the terms of order 2^-8 NP and below
// are dropped), accumulated in one float32 accumulator:
//   NP = 2:  x0 y0 + x0 y1 + x1 y0
//   NP = 3:  x0 y0 + x0 y1 + x1 y0 + x0 y2 + x1 y1 + x2 y0
// The six-product BF16 form is the bfloat16 scheme of Henry, Tang and
// Heinecke (ARITH 2019): float32-level products that keep float32's exponent
// range.  For FP16 the fixed shift k = 14 puts the largest entry of a
// normalised matrix (||X'||_F < 2^15) inside FP16 range and keeps typical
// entries, and their second parts, well above FP16's subnormals (an entry of
// size 2^-12, the typical one of a normalised 4096 x 4096 matrix, becomes 4
// and its second part about 2^-10).  BF16 has float32's exponent range and
// needs no shift.  One accumulator instead of one per order of magnitude
// halves the accumulator registers, which lets two waves share a SIMD.
//
// split_kernel turns a float32 matrix into its parts in two layouts:
// row-major (the left operand: a lane reads 8 consecutive k of its row) and
// transposed (the right operand: row j holds column j, so a lane again reads
// 8 consecutive k).  Both are zero-padded to ld = n rounded up to 256, so the
// product kernel's loads need no bounds checks.
#include <type_traits>

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

// One 64 x 64 tile per workgroup.  The tile's float32 loads are issued before
// the partial sums of squares are reduced, so the two latencies overlap.  A
// thread holds two runs of 8 entries of one row (rows tid/8 and tid/8 + 32,
// columns 8 (tid % 8) ...), writes their row-major parts as 16-byte stores
// and the scaled floats to an LDS tile padded to 65 columns; it then reads 8
// consecutive rows of one column (rows 8 (tid % 8) ..., columns tid/8 and
// tid/8 + 32) and writes their transposed parts, again as 16-byte stores.
// With the padding, the word addresses of a wave's 64 lanes fall in 64
// distinct banks in both LDS passes (the compiler pairs two words per lane
// into one access, which then takes two cycles).  Every part is a function of the scaled entry alone, so both layouts
// hold the same values.
template <typename T, int NP>
__global__ __launch_bounds__(256) void split_kernel(SplitLaunch s) {
    typedef SplitTraits<T> Tr;
    typedef typename Vec8<T>::type V8;
    __shared__ double red[256];
    __shared__ float tile[STS][STS + 1];
    const int tid = threadIdx.x;
    const int n = s.n, ld = s.ld;
    const int r0 = blockIdx.y * STS, c0 = blockIdx.x * STS;
    const bool vec = (n % 4) == 0 && ((uintptr_t)s.X & 15) == 0;
    const int lr = tid / 8, lc = (tid % 8) * 8;

    float v[2][8];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int gr = r0 + lr + 32 * q, gc = c0 + lc;
#pragma unroll
        for (int t = 0; t < 8; ++t) v[q][t] = 0.f;
        if (gr < n) {
            const float *row = s.X + (int64_t)gr * n;
            if (vec && gc + 7 < n) {
                const f4 a = *(const f4 *)(row + gc), b = *(const f4 *)(row + gc + 4);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    v[q][t] = a[t];
                    v[q][t + 4] = b[t];
                }
            } else {
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (gc + t < n) v[q][t] = row[gc + t];
            }
        }
    }

    const int eX = exponent_of_sumsq(sum_partials<256>(s.part, s.nPart, red));
    if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0 && s.eSlot) *s.eSlot = eX;
    const PowScale f = pow2_neg(eX - Tr::kShift);

#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int r = lr + 32 * q;
        V8 pv[NP];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            float x = v[q][t] * f.a * f.b;
            tile[r][lc + t] = x;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const T h = (T)x;
                pv[k][t] = h;
                x = x - (float)h;  // exact: the rest of x after the first k + 1 parts
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) *(V8 *)((T *)s.rm[k] + (int64_t)(r0 + r) * ld + c0 + lc) = pv[k];
    }
    __syncthreads();
    const int tr0 = (tid % 8) * 8;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int c = tid / 8 + 32 * q;
        V8 pv[NP];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            float x = tile[tr0 + t][c];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const T h = (T)x;
                pv[k][t] = h;
                x = x - (float)h;
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) *(V8 *)((T *)s.tr[k] + (int64_t)(c0 + c) * ld + r0 + tr0) = pv[k];
    }
}

// ------------------------------------------------------------------ product

// Operand exponents of a product whose operands' parts are those of
// unnormalised matrices (the fused split): from the producers' partial sums,
// reduced by each wave on its own (no barrier); 0 for an operand without
// partial sums.  Block 0 records eX.
struct SplitExps {
    int x, y;
};
__device__ __forceinline__ SplitExps split_operand_exps(const SplitGemmLaunch &g) {
    SplitExps e{0, 0};
    if (g.partX) e.x = exponent_of_sumsq(wave_sum_partials(g.partX, g.nPartX));
    if (g.partY) e.y = g.partY == g.partX ? e.x : exponent_of_sumsq(wave_sum_partials(g.partY, g.nPartY));
    if (g.eSlot && blockIdx.x == 0 && threadIdx.x == 0) *g.eSlot = e.x;
    return e;
}

// Epilogue of a split product tile: v = acc * 2^-2k (and * 2^-(eX + eY) for
// the fused split, both exact powers of two); the tile's float64 sum of
// squares of the valid v goes to partC[blockIdx.x].  The wave's block of
// (32 FM) x (32 FN) values starts at (m0w, n0w).  Then either v is stored to
// C, or (PARTS, g.prm and g.ptr set) v's NP 16-bit parts are, row-major and transposed,
// for the next product: v = x0 + x1 (+ x2) as split_kernel forms them, on
// the tile's whole area (its rows and columns past n hold zeros, which keeps
// the zero padding the next product reads).  `red` holds NW doubles.
template <typename T, int NP, int FM, int FN, int NW, bool PARTS>
__device__ __forceinline__ void split_epilogue(const v16f (&acc)[FM][FN], const SplitGemmLaunch &g,
                                               int m0w, int n0w, SplitExps ex, double *red) {
    typedef SplitTraits<T> Tr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 5, l32 = lane & 31;
    const int n = g.n, ld = g.ld;
    const float outScale = ldexpf(1.0f, -2 * Tr::kShift);
    const bool fused = ex.x + ex.y != 0;
    const PowScale f = pow2_neg(ex.x + ex.y);
    double ss = 0.0;
    typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            // transposed parts of rows 8 rb + 4 grp .. + 3 of column col
            u16x4 wt[PARTS ? NP : 1][4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
                const int row0 = m0w + i * 32 + 8 * rb + 4 * grp;
                const int col = n0w + j * 32 + l32;
                float v[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    v[t] = acc[i][j][4 * rb + t] * outScale;
                    if (fused) v[t] = v[t] * f.a * f.b;
                    if (row0 + t < n && col < n) ss += (double)v[t] * (double)v[t];
                }
                if constexpr (PARTS) {
                    T pv[NP][4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        float x = v[t];
#pragma unroll
                        for (int k = 0; k < NP; ++k) {
                            const T h = (T)x;
                            pv[k][t] = h;
                            x = x - (float)h;  // exact: the rest after k + 1 parts
                        }
                    }
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        T *rm = (T *)g.prm[k];
#pragma unroll
                        for (int t = 0; t < 4; ++t) rm[(int64_t)(row0 + t) * ld + col] = pv[k][t];
#pragma unroll
                        for (int t = 0; t < 4; ++t) wt[k][rb][t] = __builtin_bit_cast(unsigned short, pv[k][t]);
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (row0 + t < n && col < n) g.C[(int64_t)(row0 + t) * n + col] = v[t];
                }
            }
            if constexpr (PARTS) {
                // Transposed parts, eight consecutive rows of column col per
                // 16-byte store: for the row groups rb and rb + 1, the lane of
                // half 0 (rows 8 rb + 0 .. 3) takes rows 8 rb + 4 .. 7 from its
                // partner in half 1, which takes rows 8 rb + 8 .. 11 in turn
                // (v_permlane32_swap: [1] reads the upper half's lane, [0] the
                // lower half's).
                const int col = n0w + j * 32 + l32;
#pragma unroll
                for (int k = 0; k < NP; ++k)
#pragma unroll
                    for (int rb = 0; rb < 4; rb += 2) {
                        typedef int i32x2 __attribute__((ext_vector_type(2)));
                        const i32x2 a = __builtin_bit_cast(i32x2, wt[k][rb]);
                        const i32x2 b = __builtin_bit_cast(i32x2, wt[k][rb + 1]);
                        // every lane takes part in the lane moves
                        i32x2 sa, sb;
                        sa[0] = __builtin_amdgcn_permlane32_swap(a[0], a[0], false, false)[1];
                        sa[1] = __builtin_amdgcn_permlane32_swap(a[1], a[1], false, false)[1];
                        sb[0] = __builtin_amdgcn_permlane32_swap(b[0], b[0], false, false)[0];
                        sb[1] = __builtin_amdgcn_permlane32_swap(b[1], b[1], false, false)[0];
                        const i32x2 mine = grp == 0 ? a : b, other = grp == 0 ? sa : sb;
                        typedef int i32x4 __attribute__((ext_vector_type(4)));
                        const i32x4 w = grp == 0 ? i32x4{mine[0], mine[1], other[0], other[1]}
                                                 : i32x4{other[0], other[1], mine[0], mine[1]};
                        const int r8 = m0w + i * 32 + 8 * rb + 8 * grp;
                        *(i32x4 *)((T *)g.ptr[k] + (int64_t)col * ld + r8) = w;
                    }
            }
        }
    ss = wave_sum_lane0(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w];
        g.partC[blockIdx.x] = t;
    }
}

// SBK is the K extent (16-bit elements) of one LDS tile; rows are padded by 8
// elements so that 16-byte LDS reads are conflict-free.
template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, bool PARTS>
__global__ __launch_bounds__(WM *WN * 64) void gemm_split_kernel(SplitGemmLaunch g) {
    typedef typename Vec8<T>::type V8;
    constexpr int SLD = SBK + 8;
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;

    __shared__ __attribute__((aligned(16))) T As[NP][2][BM * SLD];
    __shared__ __attribute__((aligned(16))) T Bs[NP][2][BN * SLD];
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
    u4 ra[NP][LA], rb[NP][LB];

    auto gload = [&](int k0) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / CPR, c = (idx % CPR) * 8;
                ra[k][r] = *(const u4 *)((const T *)g.x[k] + (int64_t)(m0 + row) * ld + k0 + c);
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / CPR, c = (idx % CPR) * 8;
                rb[k][r] = *(const u4 *)((const T *)g.y[k] + (int64_t)(n0 + row) * ld + k0 + c);
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / CPR, c = (idx % CPR) * 8;
                *(u4 *)(&As[k][buf][row * SLD + c]) = ra[k][r];
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / CPR, c = (idx % CPR) * 8;
                *(u4 *)(&Bs[k][buf][row * SLD + c]) = rb[k][r];
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

    // m0 / n0 rows beyond n read the zero padding (ld is a multiple of 256).
    const int nk = (n + SBK - 1) / SBK;
    gload(0);
    const SplitExps ex = split_operand_exps(g);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * SBK);
#pragma unroll
        for (int s = 0; s < SBK / 16; ++s) {
            V8 a[NP][FM], b[NP][FN];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    a[k][i] = *(const V8 *)(&As[k][cur][(wm * TM + i * 32 + l32) * SLD + s * 16 + grp * 8]);
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[k][j] = *(const V8 *)(&Bs[k][cur][(wn * TN + j * 32 + l32) * SLD + s * 16 + grp * 8]);
            }
            // per accumulator, in this fixed order: the products x_u y_v
            // grouped by d = u + v = 0, 1, ..., NP - 1, u ascending within a
            // group: x0y0, x0y1, x1y0 (, x0y2, x1y1, x2y0)
#pragma unroll
            for (int d = 0; d < NP; ++d)
#pragma unroll
                for (int u = 0; u <= d; ++u)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = mfma16<T>(a[u][i], b[d - u][j], acc[i][j]);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    split_epilogue<T, NP, FM, FN, WM * WN, PARTS>(acc, g, m0 + wm * TM, n0 + wn * TN, ex, red);
}

template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, bool PARTS>
hipError_t launch_gemm_split(const SplitGemmLaunch &g, hipStream_t s) {
    const int tiles = ((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    hipLaunchKernelGGL((gemm_split_kernel<T, NP, BM, BN, WM, WN, SBK, PARTS>), dim3(tiles),
                       dim3(WM * WN * 64), 0, s, g);
    return hipGetLastError();
}

// The same product with its operand tiles moved by LDS-DMA buffer loads
// (global -> LDS without VGPRs; lane l of a load lands at byte 16 l of a
// 1 KB LDS window).  The parts are zero-padded ld x ld arrays, so a tile
// never needs a bounds check, and the K advance is the loads' scalar offset.
// LDS rows are unpadded (SBK 16-bit elements); 16-byte chunk c of row r sits
// at chunk position c ^ swz(r), which spreads the rows that share LDS banks
// (rows r + 16/CPR apart) over distinct positions, so the 16-byte operand
// reads are conflict-free.  Without padding a 256 x 256 tile with SBK = 32
// fits LDS twice (double buffer), halving the barriers of the SBK = 16
// register-staged tile.  Products per 16-wide K chunk in the same order as
// gemm_split_kernel: bit-identical results.  Needs ld <= kSplitDmaMaxLd.
template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, bool PARTS>
__global__ __launch_bounds__(WM *WN * 64) void gemm_split_dma_kernel(SplitGemmLaunch g) {
    typedef typename Vec8<T>::type V8;
    constexpr int NT = WM * WN * 64, NW = NT / 64;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int CPR = SBK / 8;   // 16-byte chunks per tile row
    constexpr int RPS = 64 / CPR;  // tile rows per 1 KB load
    constexpr int A_PER = BM / RPS / NW, B_PER = BN / RPS / NW;  // loads per wave and part
    static_assert(A_PER * NW * RPS == BM && B_PER * NW * RPS == BN && A_PER > 0 && B_PER > 0,
                  "loads");
    // two buffers as separate arrays, so the compiler sees that the loads
    // into one do not alias the operand reads from the other
    __shared__ __attribute__((aligned(16))) T A0[NP][BM * SBK];
    __shared__ __attribute__((aligned(16))) T A1[NP][BM * SBK];
    __shared__ __attribute__((aligned(16))) T B0[NP][BN * SBK];
    __shared__ __attribute__((aligned(16))) T B1[NP][BN * SBK];
    __shared__ double red[NW];

    const int n = g.n, ld = g.ld;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN, grp = lane >> 5, l32 = lane & 31;
    int tm, tn;
    tile_of_block(blockIdx.x, (n + BM - 1) / BM, (n + BN - 1) / BN, &tm, &tn);
    const int m0 = tm * BM, n0 = tn * BN;
    auto swz = [](int row) { return (row / (16 / CPR)) % CPR; };
    typedef __attribute__((address_space(3))) void lds_void;
    const int bytes = ld * ld * 2;
    __amdgpu_buffer_rsrc_t rx[NP], ry[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        rx[k] = __builtin_amdgcn_make_buffer_rsrc((void *)g.x[k], (short)0, bytes, 0x00020000);
        ry[k] = __builtin_amdgcn_make_buffer_rsrc((void *)g.y[k], (short)0, bytes, 0x00020000);
    }
    unsigned a_off[A_PER], b_off[B_PER];
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
        const int row = RPS * (wave + r * NW) + lane / CPR;
        a_off[r] = (unsigned)(((m0 + row) * ld + 8 * ((lane % CPR) ^ swz(row))) * 2);
    }
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
        const int row = RPS * (wave + r * NW) + lane / CPR;
        b_off[r] = (unsigned)(((n0 + row) * ld + 8 * ((lane % CPR) ^ swz(row))) * 2);
    }
    auto load_tile = [&](int k0, T (*as)[BM * SBK], T (*bs)[BN * SBK]) {
        const unsigned so = (unsigned)(k0 * 2);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
#pragma unroll
            for (int r = 0; r < A_PER; ++r) {
                const unsigned off = a_off[r];
                const __amdgpu_buffer_rsrc_t rr = rx[k];
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rr, (lds_void *)(as[k] + (wave + r * NW) * 512), 16, off, so, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < B_PER; ++r) {
                const unsigned off = b_off[r];
                const __amdgpu_buffer_rsrc_t rr = ry[k];
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rr, (lds_void *)(bs[k] + (wave + r * NW) * 512), 16, off, so, 0, 0);
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

    // m0 / n0 rows beyond n read the zero padding (ld is a multiple of 256).
    const int nk = (n + SBK - 1) / SBK;
    auto body = [&](int kt, T (*as)[BM * SBK], T (*bs)[BN * SBK], T (*an)[BM * SBK],
                    T (*bn)[BN * SBK]) {
        if (kt + 1 < nk) load_tile((kt + 1) * SBK, an, bn);
#pragma unroll
        for (int s = 0; s < SBK / 16; ++s) {
            V8 a[NP][FM], b[NP][FN];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int row = wm * TM + i * 32 + l32;
                    a[k][i] = *(const V8 *)(&as[k][row * SBK + 8 * ((2 * s + grp) ^ swz(row))]);
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int row = wn * TN + j * 32 + l32;
                    b[k][j] = *(const V8 *)(&bs[k][row * SBK + 8 * ((2 * s + grp) ^ swz(row))]);
                }
            }
            // the fixed product order of gemm_split_kernel
#pragma unroll
            for (int d = 0; d < NP; ++d)
#pragma unroll
                for (int u = 0; u <= d; ++u)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = mfma16<T>(a[u][i], b[d - u][j], acc[i][j]);
        }
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the next tile is in LDS
        __syncthreads();
    };
    load_tile(0, A0, B0);
    const SplitExps ex = split_operand_exps(g);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    for (int kt = 0; kt < nk; kt += 2) {
        body(kt, A0, B0, A1, B1);
        if (kt + 1 < nk) body(kt + 1, A1, B1, A0, B0);
    }
    split_epilogue<T, NP, FM, FN, NW, PARTS>(acc, g, m0 + wm * TM, n0 + wn * TN, ex, red);
}

// One 16-byte-per-lane buffer load into LDS (lane l's 16 bytes land at byte
// lds + 16 l), written as assembly: the compiler then keeps no count of these
// loads and inserts no waits for them, and the kernel that issues them waits
// for them itself.  The LDS address goes through m0, which the sequence saves
// and restores; one wait state separates the m0 write from the load that
// reads it.  rsrc is a raw buffer descriptor (base, stride 0, num_records =
// bytes, so an offset past the end reads zeros).
__device__ __forceinline__ void lds_load16_asm(u4 rsrc, unsigned lds, unsigned voff,
                                               unsigned soff) {
    unsigned saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %1\n\t"
        "s_nop 0\n\t"
        "buffer_load_dwordx4 %2, %3, %4 offen lds\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "s"(lds), "v"(voff), "s"(rsrc), "s"(soff)
        : "memory");
}

// vmcnt(N) alone (expcnt and lgkmcnt left at their maxima), for s_waitcnt.
constexpr int vmcnt_only(int N) { return 0x0f70 | (N & 15) | ((N >> 4) << 14); }

// Multi-stage form of gemm_split_dma_kernel: NS (3 or 4) LDS buffers.  While
// tile kt is multiplied, the loads of tiles kt + 1 ... kt + NS - 1 are in
// flight, so a tile's load has NS - 1 tiles of MFMA work to arrive in, where
// the two-buffer kernel gives it one.  A workgroup barrier made by
// __syncthreads() also waits for every outstanding load (vmcnt(0)), which
// would cap the depth at one tile, so each wave instead waits only for its
// own loads of tile kt (vmcnt = the loads of the NS - 2 later tiles, counted
// at compile time) and then meets the others at a bare s_barrier.  The loads
// of the tile issued at step kt go to the buffer read at step kt - 1, which
// every wave has left by the time it passes step kt's barrier.  Past the last
// tile the loads repeat tile 0 into buffers that are never read, so that the
// count of loads in flight is the same at every step.  Same operand layout,
// loads and per-16-wide-K product order as gemm_split_dma_kernel:
// bit-identical results.  Needs ld <= kSplitDmaMaxLd.
template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, int NS, bool PARTS>
__global__ __launch_bounds__(WM *WN * 64) void gemm_split_ms_kernel(SplitGemmLaunch g) {
    static_assert(NS == 3 || NS == 4, "stages");
    typedef typename Vec8<T>::type V8;
    constexpr int NT = WM * WN * 64, NW = NT / 64;
    constexpr int TM = BM / WM, TN = BN / WN, FM = TM / 32, FN = TN / 32;
    constexpr int CPR = SBK / 8;   // 16-byte chunks per tile row
    constexpr int RPS = 64 / CPR;  // tile rows per 1 KB load
    constexpr int A_PER = BM / RPS / NW, B_PER = BN / RPS / NW;  // loads per wave and part
    static_assert(A_PER * NW * RPS == BM && B_PER * NW * RPS == BN && A_PER > 0 && B_PER > 0,
                  "loads");
    constexpr int LPT = NP * (A_PER + B_PER);  // loads per lane and tile
    static_assert((NS - 2) * LPT <= 63, "vmcnt range");
    constexpr int AS = BM * SBK, BS = BN * SBK, SS = NP * (AS + BS);
    // one array per stage (the parts of X, then those of Y): the compiler
    // tracks which LDS array each load writes, for only a few arrays, and
    // then sees that the loads into one stage do not alias the operand reads
    // from another
    __shared__ __attribute__((aligned(16))) T S0[SS];
    __shared__ __attribute__((aligned(16))) T S1[SS];
    __shared__ __attribute__((aligned(16))) T S2[SS];
    __shared__ __attribute__((aligned(16))) T S3[NS > 3 ? SS : 8];
    __shared__ double red[NW];

    const int n = g.n, ld = g.ld;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN, grp = lane >> 5, l32 = lane & 31;
    int tm, tn;
    tile_of_block(blockIdx.x, (n + BM - 1) / BM, (n + BN - 1) / BN, &tm, &tn);
    const int m0 = tm * BM, n0 = tn * BN;
    auto swz = [](int row) { return (row / (16 / CPR)) % CPR; };
    const unsigned bytes = (unsigned)ld * (unsigned)ld * 2u;
    auto rsrc = [&](const void *p) {
        const uint64_t a = (uint64_t)(uintptr_t)p;
        u4 r;
        r[0] = (unsigned)a;
        r[1] = (unsigned)(a >> 32) & 0xffffu;  // stride 0
        r[2] = bytes;
        r[3] = 0x00020000u;
        return r;
    };
    u4 rx[NP], ry[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        rx[k] = rsrc(g.x[k]);
        ry[k] = rsrc(g.y[k]);
    }
    unsigned a_off[A_PER], b_off[B_PER];
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
        const int row = RPS * (wave + r * NW) + lane / CPR;
        a_off[r] = (unsigned)(((m0 + row) * ld + 8 * ((lane % CPR) ^ swz(row))) * 2);
    }
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
        const int row = RPS * (wave + r * NW) + lane / CPR;
        b_off[r] = (unsigned)(((n0 + row) * ld + 8 * ((lane % CPR) ^ swz(row))) * 2);
    }
    auto load_tile = [&](int k0, T *st) {
        const unsigned so = (unsigned)(k0 * 2);
        const unsigned base = (unsigned)(uintptr_t)(__attribute__((address_space(3))) T *)st;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
#pragma unroll
            for (int r = 0; r < A_PER; ++r)
                lds_load16_asm(rx[k], base + 2u * (unsigned)(k * AS + (wave + r * NW) * 512), a_off[r],
                               so);
#pragma unroll
            for (int r = 0; r < B_PER; ++r)
                lds_load16_asm(ry[k],
                               base + 2u * (unsigned)(NP * AS + k * BS + (wave + r * NW) * 512),
                               b_off[r], so);
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
    auto body = [&](int kt, const T *st, T *nx) {
        __builtin_amdgcn_s_waitcnt(vmcnt_only((NS - 2) * LPT));  // this lane's loads of tile kt
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        const int kl = kt + NS - 1;
        load_tile(kl < nk ? kl * SBK : 0, nx);
#pragma unroll
        for (int s = 0; s < SBK / 16; ++s) {
            V8 a[NP][FM], b[NP][FN];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int row = wm * TM + i * 32 + l32;
                    a[k][i] = *(const V8 *)(st + k * AS + row * SBK + 8 * ((2 * s + grp) ^ swz(row)));
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int row = wn * TN + j * 32 + l32;
                    b[k][j] = *(const V8 *)(st + NP * AS + k * BS + row * SBK + 8 * ((2 * s + grp) ^ swz(row)));
                }
            }
#pragma unroll
            for (int d = 0; d < NP; ++d)
#pragma unroll
                for (int u = 0; u <= d; ++u)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = mfma16<T>(a[u][i], b[d - u][j], acc[i][j]);
        }
    };
    load_tile(0, S0);
    load_tile(1 < nk ? SBK : 0, S1);
    if constexpr (NS > 3) load_tile(2 < nk ? 2 * SBK : 0, S2);
    const SplitExps ex = split_operand_exps(g);
    for (int kt = 0; kt < nk; kt += NS) {
        if constexpr (NS > 3) {
            body(kt, S0, S3);
            if (kt + 1 < nk) body(kt + 1, S1, S0);
            if (kt + 2 < nk) body(kt + 2, S2, S1);
            if (kt + 3 < nk) body(kt + 3, S3, S2);
        } else {
            body(kt, S0, S2);
            if (kt + 1 < nk) body(kt + 1, S1, S0);
            if (kt + 2 < nk) body(kt + 2, S2, S1);
        }
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_only(0));  // no LDS write still in flight at exit
    split_epilogue<T, NP, FM, FN, NW, PARTS>(acc, g, m0 + wm * TM, n0 + wn * TN, ex, red);
}

// Largest ld whose ld x ld 16-bit part a 32-bit buffer offset covers
// (a multiple of 256 with ld^2 * 2 < 2^31).
constexpr int kSplitDmaMaxLd = 32512;

// The LDS-DMA kernel when the padded parts fit a buffer's range (two LDS
// buffers for DNS = 2, gemm_split_ms_kernel with DNS stages otherwise), else
// the register-staged one of the same tile (same results in every case).
template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, int DWM, int DWN,
          int DSBK, int DNS, bool PARTS>
hipError_t launch_split_product_as(const SplitGemmLaunch &g, hipStream_t s) {
    if (g.ld > kSplitDmaMaxLd) return launch_gemm_split<T, NP, BM, BN, WM, WN, SBK, PARTS>(g, s);
    const int tiles = ((g.n + BM - 1) / BM) * ((g.n + BN - 1) / BN);
    if constexpr (DNS == 2)
        hipLaunchKernelGGL((gemm_split_dma_kernel<T, NP, BM, BN, DWM, DWN, DSBK, PARTS>),
                           dim3(tiles), dim3(DWM * DWN * 64), 0, s, g);
    else
        hipLaunchKernelGGL((gemm_split_ms_kernel<T, NP, BM, BN, DWM, DWN, DSBK, DNS, PARTS>),
                           dim3(tiles), dim3(DWM * DWN * 64), 0, s, g);
    return hipGetLastError();
}

// The instance that writes the result's parts (the fused split; BF16 only)
// when g.prm is set, else the one that writes the float32 result.
template <typename T, int NP, int BM, int BN, int WM, int WN, int SBK, int DWM, int DWN,
          int DSBK, int DNS>
hipError_t launch_split_product(const SplitGemmLaunch &g, hipStream_t s) {
    if constexpr (std::is_same<T, __bf16>::value) {
        if (g.prm[0])
            return launch_split_product_as<T, NP, BM, BN, WM, WN, SBK, DWM, DWN, DSBK, DNS, true>(g, s);
    } else {
        if (g.prm[0]) return hipErrorInvalidValue;  // FP16 parts need the scale first
    }
    return launch_split_product_as<T, NP, BM, BN, WM, WN, SBK, DWM, DWN, DSBK, DNS, false>(g, s);
}

}  // namespace

int split_parts(int mode) { return mode == MPOW_BF16X6 ? 3 : (mode == MPOW_FP32 ? 0 : 2); }

// Padded leading dimension of the split operands: a multiple of the largest
// product tile, so tiles read zeros past n and need no bounds checks.
int split_ld(int n) { return (n + 255) / 256 * 256; }

hipError_t launch_split(int mode, const SplitLaunch &sl, hipStream_t s) {
    const dim3 grid(sl.ld / STS, sl.ld / STS);
    if (mode == MPOW_FP16X3)
        hipLaunchKernelGGL((split_kernel<_Float16, 2>), grid, dim3(256), 0, s, sl);
    else if (mode == MPOW_BF16X3)
        hipLaunchKernelGGL((split_kernel<__bf16, 2>), grid, dim3(256), 0, s, sl);
    else if (mode == MPOW_BF16X6)
        hipLaunchKernelGGL((split_kernel<__bf16, 3>), grid, dim3(256), 0, s, sl);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// 256 x 256 or 128 x 128 tiles, whichever has the higher estimated rate:
// the rate for how its tile count fills the CUs (tile_fill_rate), with
// full-wave rates measured on MI355X (16-bit MFMA TFLOP/s, LDS-DMA kernels):
// X3 modes (4 x 2 waves) 256 x 256 1250, 128 x 128 1040; BF16X6 (three-stage
// kernels) 1270 and 1110, times the useful fraction of the padded output
// area, (n / (tiles per side x edge))^2, so that a small matrix (n <= 128:
// one tile either way) takes the tile with less padding.  Both accumulate
// every output in the same order (per 16-wide K chunk, the fixed product
// order above), so the two give bit-identical results.
static double split_rate(double full_wave, int n, int edge) {
    const int t = (n + edge - 1) / edge;
    const double useful = (double)n / (double)(t * edge);
    return tile_fill_rate(full_wave, n, edge, edge) * useful * useful;
}

int gemm_split_pick(int mode, int n) {
    const bool x6 = mode == MPOW_BF16X6;
    const bool big = split_rate(x6 ? 1270.0 : 1250.0, n, 256) > split_rate(x6 ? 1110.0 : 1040.0, n, 128);
    if (mode == MPOW_FP16X3) return big ? MPOW_KERNEL_GEMM_F16X3_256 : MPOW_KERNEL_GEMM_F16X3_128;
    if (x6) return big ? MPOW_KERNEL_GEMM_BF16X6_256 : MPOW_KERNEL_GEMM_BF16X6_128;
    return big ? MPOW_KERNEL_GEMM_BF16X3_256 : MPOW_KERNEL_GEMM_BF16X3_128;
}

int gemm_split_mode(int kernel) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F16X3_128:
        case MPOW_KERNEL_GEMM_F16X3_256: return MPOW_FP16X3;
        case MPOW_KERNEL_GEMM_BF16X3_128:
        case MPOW_KERNEL_GEMM_BF16X3_256: return MPOW_BF16X3;
        case MPOW_KERNEL_GEMM_BF16X6_128:
        case MPOW_KERNEL_GEMM_BF16X6_256: return MPOW_BF16X6;
        default: return -1;
    }
}

static int split_tile_edge(int kernel) {
    return (kernel == MPOW_KERNEL_GEMM_F16X3_256 || kernel == MPOW_KERNEL_GEMM_BF16X3_256 ||
            kernel == MPOW_KERNEL_GEMM_BF16X6_256)
               ? 256
               : 128;
}

int gemm_split_tiles(int kernel, int n) {
    const int e = split_tile_edge(kernel);
    const int t = (n + e - 1) / e;
    return t * t;
}

const char *gemm_split_name(int kernel) {
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F16X3_128: return "gemm_split_dma_kernel<_Float16,2,128,128,4,2,64>";
        case MPOW_KERNEL_GEMM_BF16X3_128: return "gemm_split_dma_kernel<__bf16,2,128,128,4,2,64>";
        case MPOW_KERNEL_GEMM_F16X3_256: return "gemm_split_dma_kernel<_Float16,2,256,256,4,2,32>";
        case MPOW_KERNEL_GEMM_BF16X3_256: return "gemm_split_dma_kernel<__bf16,2,256,256,4,2,32>";
        case MPOW_KERNEL_GEMM_BF16X6_128: return "gemm_split_ms_kernel<__bf16,3,128,128,2,4,32,3>";
        case MPOW_KERNEL_GEMM_BF16X6_256: return "gemm_split_ms_kernel<__bf16,3,256,256,2,4,16,3>";
        default: return nullptr;
    }
}

hipError_t gemm_split_launch(int kernel, const SplitGemmLaunch &g, hipStream_t s) {
    // register-staged tile <BM, BN, WM, WN, SBK>, then the LDS-DMA waves, K tile
    // and stages
    switch (kernel) {
        case MPOW_KERNEL_GEMM_F16X3_128:
            return launch_split_product<_Float16, 2, 128, 128, 2, 2, 32, 4, 2, 64, 2>(g, s);
        case MPOW_KERNEL_GEMM_BF16X3_128:
            return launch_split_product<__bf16, 2, 128, 128, 2, 2, 32, 4, 2, 64, 2>(g, s);
        case MPOW_KERNEL_GEMM_F16X3_256:
            return launch_split_product<_Float16, 2, 256, 256, 2, 4, 16, 4, 2, 32, 2>(g, s);
        case MPOW_KERNEL_GEMM_BF16X3_256:
            return launch_split_product<__bf16, 2, 256, 256, 2, 4, 16, 4, 2, 32, 2>(g, s);
        case MPOW_KERNEL_GEMM_BF16X6_128:
            return launch_split_product<__bf16, 3, 128, 128, 2, 2, 32, 2, 4, 32, 3>(g, s);
        case MPOW_KERNEL_GEMM_BF16X6_256:
            return launch_split_product<__bf16, 3, 256, 256, 2, 4, 16, 2, 4, 16, 3>(g, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mpow
