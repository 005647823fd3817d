// One BM x BN output tile of the float32 product C = (2^-eX X)(2^-eY Y)
// whose operand tiles stream from memory straight into LDS (the paper's
// tiled product, section 4.3.7, with the tiles kept consistent by barriers,
// section 4.3.6).
//
// CDNA4 design (the tiles for n where the MFMA pipes are the bound):
//  - Buffer loads with the LDS-DMA form write each 16-byte chunk of the X
//    (BM x BK) and Y (BK x BN) tiles into LDS without passing through
//    VGPRs: no staging registers, no LDS store instructions, no per-element
//    arithmetic on the way.  Lane l of a wave's load lands at byte 16 l of a
//    1 KB LDS window, so the choice of which global chunk each lane fetches
//    sets the LDS layout.  Out-of-range lanes get an offset beyond the
//    buffer's range, which the hardware check turns into zeros (ragged
//    edges).  The K advance of interior tiles is a scalar offset, so issuing
//    a tile's loads costs no vector instructions.
//  - Layouts are unpadded and XOR-swizzled so that the MFMA operand reads
//    are free of LDS bank conflicts: in the X tile, 16-byte chunk c of row r
//    sits at chunk position c ^ ((r >> 1) & 7) (BK = 32) or c ^ (r & 15)
//    (BK = 64); in the Y tile, rows k with bit 4 set swap their 32-float
//    column halves.
//  - Two LDS buffers (four separate arrays) alternate: the next K tile
//    streams into one while the MFMAs read the other, one barrier per tile.
//    BK = 64 (the batched kernel's 64 x 64 tile) halves the barriers and is
//    consumed as two 32-wide halves in order; the single-matrix tiles use
//    BK = 32, whose smaller LDS footprint lets more workgroups share a CU
//    (measured faster for the 64 x 64 and 128 x 128 tiles from n = 1536 on).
//  - v_mfma_f32_32x32x2_f32, each wave a (BM/WM) x (BN/WN) block of C, with
//    the k-to-lane mapping and K order of f32_tile (K in steps of 32, lane
//    half h taking k = 16h + 4q + t of each step), so every output element
//    is accumulated in the same order as by the other float32 tiles.
//  - The power-of-two operand scales: when eX + eY lies in [-32, 96] the
//    unscaled product cannot leave the normal float range (|X Y| <=
//    ||X||_F ||Y||_F < 2^(eX+eY+2)), so the factor 2^-(eX+eY) is applied
//    once to each result in the epilogue; otherwise it is applied to the
//    operand registers after each LDS read, as f32_tile applies it on load.
//    Multiplying by a power of two is exact for normal floats and commutes
//    with every rounding of the accumulation, so both forms give the bits of
//    f32_tile wherever no product or partial sum is subnormal.
#pragma once

#include "gemm_f32_tile.h"
#include "scale_device.h"

namespace mpow {

// Largest n whose n x n float32 matrix a 32-bit buffer offset covers
// (n^2 * 4 < 2^31).
constexpr int DMA_MAX_N = 23170;

typedef __attribute__((address_space(3))) void lds_void_t;

// Compile-time flag passed to the K loop's generic lambda.
template <bool B>
struct DmaBool {
    static constexpr bool value = B;
};

// Operand exponents of one product.
struct OperandExps {
    int x, y;
};

// All WM * WN * 64 threads must call it.  `As0`/`As1` hold BM * BK floats
// each, `Bs0`/`Bs1` BK * BN floats each (four distinct LDS arrays), `red`
// WM * WN doubles.  `exps()` is called by every thread once, while
// the first tile's loads are in flight; it may contain barriers.  Requires
// n % 4 == 0, X and Y 16-byte aligned, n <= DMA_MAX_N.  Returns the tile's
// float64 sum of squares of C in thread 0 (0 elsewhere).
template <int BM, int BN, int WM, int WN, int BK, bool AXPI, typename ExpFn>
__device__ __forceinline__ double f32_tile_dma(const float *__restrict__ X,
                                               const float *__restrict__ Y, ExpFn exps,
                                               float *__restrict__ C, int n, int m0, int n0,
                                               float *As0, float *As1, float *Bs0, float *Bs1,
                                               double *red, float alpha = 1.0f) {
    static_assert(BK == 32 || BK == 64, "LDS K extent");
    constexpr int NW = WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;
    static_assert(FM * 32 == TM && FN * 32 == TN && BN >= 64, "wave tile");
    constexpr int KH = 16;                                // k per lane half and 32-step
    constexpr int ABUF = BM * BK, BBUF = BK * BN;         // floats per tile buffer
    constexpr int A_PER = ABUF / 256 / NW;                // 1 KB loads per wave, X tile
    constexpr int B_PER = BBUF / 256 / NW;                // 1 KB loads per wave, Y tile
    static_assert(A_PER * 256 * NW == ABUF && B_PER * 256 * NW == BBUF, "loads");
    constexpr int CPA = BK / 4;    // 16-byte chunks per X tile row
    constexpr int CPB = BN / 4;    // 16-byte chunks per Y tile row
    constexpr int RPB = 256 / BN;  // Y tile rows per 1 KB load

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, l32 = lane & 31;
    auto swz = [](int r) { return BK == 32 ? ((r >> 1) & 7) : (r & 15); };

    const int bytes = n * n * 4;
    const __amdgpu_buffer_rsrc_t rX =
        __builtin_amdgcn_make_buffer_rsrc((void *)X, (short)0, bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rY =
        __builtin_amdgcn_make_buffer_rsrc((void *)Y, (short)0, bytes, 0x00020000);
    constexpr unsigned OUT = 0x80000000u;  // beyond any buffer range: reads 0

    // The lane's chunk of each 1 KB load (g = wave + r NW): X load r covers
    // tile rows (256 / BK) g ..., Y load r covers tile rows RPB g ....
    int a_row[A_PER], a_col[A_PER], b_row[B_PER], b_col[B_PER];
    unsigned a_off[A_PER], b_off[B_PER];
#pragma unroll
    for (int r = 0; r < A_PER; ++r) {
        const int row = (256 / BK) * (wave + r * NW) + lane / CPA;
        a_row[r] = m0 + row;
        a_col[r] = 4 * ((lane % CPA) ^ swz(row));
        a_off[r] = a_row[r] < n ? (unsigned)((a_row[r] * n + a_col[r]) * 4) : OUT;
    }
#pragma unroll
    for (int r = 0; r < B_PER; ++r) {
        const int row = RPB * (wave + r * NW) + lane / CPB;
        b_row[r] = row;
        b_col[r] = n0 + 4 * ((lane % CPB) ^ (8 * ((row >> 4) & 1)));
        b_off[r] = b_col[r] < n ? (unsigned)((row * n + b_col[r]) * 4) : OUT;
    }
    // K tile at k0 into (as, bs).  Interior tiles: fixed lane offsets plus
    // a scalar K offset; the last, partial tile checks every chunk.
    auto load_tile = [&](int k0, float *as, float *bs) {
        if (k0 + BK <= n) {
#pragma unroll
            for (int r = 0; r < A_PER; ++r) {
                const unsigned off = a_off[r], so = (unsigned)(k0 * 4);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rX, (lds_void_t *)(as + (wave + r * NW) * 256), 16, off, so, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < B_PER; ++r) {
                const unsigned off = b_off[r], so = (unsigned)(k0 * n * 4);
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rY, (lds_void_t *)(bs + (wave + r * NW) * 256), 16, off, so, 0, 0);
            }
        } else {
#pragma unroll
            for (int r = 0; r < A_PER; ++r) {
                const int gc = k0 + a_col[r];
                const unsigned off =
                    (a_row[r] < n && gc < n) ? (unsigned)((a_row[r] * n + gc) * 4) : OUT;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rX, (lds_void_t *)(as + (wave + r * NW) * 256), 16, off, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < B_PER; ++r) {
                const int gr = k0 + b_row[r];
                const unsigned off =
                    (gr < n && b_col[r] < n) ? (unsigned)((gr * n + b_col[r]) * 4) : OUT;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(
                    rY, (lds_void_t *)(bs + (wave + r * NW) * 256), 16, off, 0, 0, 0);
            }
        }
    };

    const int nk = (n + BK - 1) / BK;
    load_tile(0, As0, Bs0);
    const OperandExps e = exps();
    const bool after = e.x + e.y >= -32 && e.x + e.y <= 96;  // scale in the epilogue
    const PowScale fx = pow2_neg(e.x), fy = pow2_neg(e.y);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's loads are in LDS
    __syncthreads();

    v16f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // K loop; SCALE_OPS scales the operand registers (the path for
    // exponents outside the epilogue-safe range).
    auto kloop = [&](auto scale_tag) {
        constexpr bool SCALE_OPS = decltype(scale_tag)::value;
        f4 a[2][FM];
        float b[2][4][FN];
        // operands of k = 32u + 16h + 4q + t, t = 0..3
        auto lds_read = [&](const float *as, const float *bs, int u, int q, int st) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int row = wm * TM + i * 32 + l32;
                a[st][i] = *(const f4 *)(as + row * BK + 4 * ((8 * u + 4 * h + q) ^ swz(row)));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int k = 32 * u + h * KH + 4 * q + t;
                    const int col = wn * TN + j * 32 + l32;
                    b[st][t][j] = bs[k * BN + (col ^ (32 * h))];
                }
        };
        constexpr int GROUPS = (BK / 32) * (KH / 4);  // groups of four k per LDS tile
        auto body = [&](int kt, const float *as, const float *bs, float *an, float *bn) {
            if (kt + 1 < nk) load_tile((kt + 1) * BK, an, bn);
            lds_read(as, bs, 0, 0, 0);
#pragma unroll
            for (int gq = 0; gq < GROUPS; ++gq) {
                const int st = gq & 1;
                if (gq + 1 < GROUPS) lds_read(as, bs, (gq + 1) / 4, (gq + 1) % 4, st ^ 1);
                if constexpr (SCALE_OPS) {
#pragma unroll
                    for (int i = 0; i < FM; ++i) a[st][i] = a[st][i] * fx.a * fx.b;
#pragma unroll
                    for (int t = 0; t < 4; ++t)
#pragma unroll
                        for (int j = 0; j < FN; ++j) b[st][t][j] = b[st][t][j] * fy.a * fy.b;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                                a[st][i][t], b[st][t][j], acc[i][j], 0, 0, 0);
            }
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): next tile is in LDS
            __syncthreads();
        };
        for (int kt = 0; kt < nk; kt += 2) {
            body(kt, As0, Bs0, As1, Bs1);
            if (kt + 1 < nk) body(kt + 1, As1, Bs1, As0, Bs0);
        }
    };
    if (after)
        kloop(DmaBool<false>{});
    else
        kloop(DmaBool<true>{});

    // 32x32 accumulator layout: register r of lane l holds row
    // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the 32x32 block.
    const PowScale fs = pow2_neg(after ? e.x + e.y : 0);
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * TM + i * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int col = n0 + wn * TN + j * 32 + l32;
                if (row < n && col < n) {
                    float v = acc[i][j][r] * fs.a * fs.b;
                    if constexpr (AXPI) v = fmaf(v, alpha, row == col ? 1.0f : 0.0f);
                    C[(int64_t)row * n + col] = v;
                    ss += (double)v * (double)v;
                }
            }
    ss = wave_sum_lane0(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double t = 0.0;
    if (tid == 0) {
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w];
    }
    __syncthreads();  // red and the LDS tiles may be reused by the caller
    return t;
}

}  // namespace mpow

namespace mpow {

// Small n (n <= DMA_K4_MAX_N): one 32 x 32 output tile per workgroup, its K
// range split over 4 waves, with the whole K range of both operand panels
// (32 x n of X, n x 32 of Y) held in LDS.  At such n a K tile's MFMAs (16
// per wave) take less time than its loads' memory latency, so a tile-by-tile
// double buffer waits on memory at every step; here every load of the tile
// is issued at once (stages of 128 values of K, each its own LDS region, 8
// LDS-DMA loads per wave and stage), the tile waits once and then runs all
// its MFMAs without a barrier.  Wave w takes the 32-wide K slices w, w + 4,
// w + 8, ... in ascending order and the four partial tiles are added in wave
// order, as the register-staged 32 x 32 tile with a 4-way K split does, so
// the two give the same products (and the operand scales are applied as in
// f32_tile_dma); their tile sums of squares are added in different float64
// orders, which can move the next exponent only for a sum within rounding
// of a power of four.  Layouts: a stage's X block is 32 rows of 128 floats, 16-byte
// chunk c of row r at position c ^ (r & 15); its Y block is 128 rows of 32
// floats, row k at float 32 k + 32 (k / 16) (a gap of 32 floats after every
// 16 rows), so the lane halves' reads (rows k and k + 16) use different LDS
// banks.
constexpr int DMA_K4_MAX_N = 512;
constexpr int DMA_K4_STAGES = DMA_K4_MAX_N / 128;
constexpr int DMA_K4_A_STAGE = 32 * 128;       // floats of one stage's X block
constexpr int DMA_K4_B_STAGE = 128 * 32 + 32 * 8;  // floats of one stage's Y block

// All KS * 64 threads must call it (KS = 4 or 8 waves: wave w takes the
// slices w, w + KS, ...).  As[s] / Bs[s] (s < DMA_K4_STAGES) are LDS arrays
// of DMA_K4_A_STAGE / DMA_K4_B_STAGE floats.  Same requirements and return
// value as f32_tile_dma, and n <= DMA_K4_MAX_N.  With KS = 8 the products
// are those of the register-staged 32 x 32 tile with an 8-way K split.
template <int KS, bool AXPI, typename ExpFn>
__device__ __forceinline__ double f32_tile_dma_k4(const float *__restrict__ X,
                                                  const float *__restrict__ Y, ExpFn exps,
                                                  float *__restrict__ C, int n, int m0, int n0,
                                                  float *const *As, float *const *Bs,
                                                  float alpha = 1.0f) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, l32 = lane & 31;
    const int bytes = n * n * 4;
    const __amdgpu_buffer_rsrc_t rX =
        __builtin_amdgcn_make_buffer_rsrc((void *)X, (short)0, bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rY =
        __builtin_amdgcn_make_buffer_rsrc((void *)Y, (short)0, bytes, 0x00020000);
    constexpr unsigned OUT = 0x80000000u;
    const int nst = (n + 127) / 128;  // stages
    const int nsl = (n + 31) / 32;    // 32-wide K slices

    static_assert(KS == 4 || KS == 8, "K split over 4 or 8 waves");
    constexpr int LPW = 16 / KS;  // loads per wave and stage, of each operand
    // Stage s: X rows m0..m0+31, K [128 s, 128 s + 128) in 16 loads of 2 rows,
    // Y rows 128 s ... in 16 loads of 8 rows; wave w issues loads LPW w ...
    // LPW w + LPW - 1 of each.
    auto load_stage = [&](int s) {
        const int k0 = 128 * s;
        float *as = As[s];
        float *bs = Bs[s];
#pragma unroll
        for (int r = 0; r < LPW; ++r) {
            const int u = LPW * wave + r;        // rows 2u, 2u + 1
            const int row = 2 * u + (lane >> 5);
            const int gc = k0 + 4 * ((lane & 31) ^ (row & 15));
            const int gr = m0 + row;
            const unsigned off = (gr < n && gc < n) ? (unsigned)((gr * n + gc) * 4) : OUT;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rX, (lds_void_t *)(as + u * 256), 16, off, 0,
                                                     0, 0);
        }
#pragma unroll
        for (int r = 0; r < LPW; ++r) {
            const int g = LPW * wave + r;        // rows 8g .. 8g + 7
            const int gr = k0 + 8 * g + (lane >> 3);
            const int gc = n0 + 4 * (lane & 7);
            const unsigned off = (gr < n && gc < n) ? (unsigned)((gr * n + gc) * 4) : OUT;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(
                rY, (lds_void_t *)(bs + g * 256 + 32 * (g >> 1)), 16, off, 0, 0, 0);
        }
    };

    // Every stage's loads at once (at most 128 KB per workgroup); one wait.
#pragma unroll
    for (int s = 0; s < DMA_K4_STAGES; ++s)
        if (s < nst) load_stage(s);
    const OperandExps e = exps();
    const bool after = e.x + e.y >= -32 && e.x + e.y <= 96;  // scale in the epilogue
    const PowScale fx = pow2_neg(e.x), fy = pow2_neg(e.y);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's loads are in LDS
    __syncthreads();

    v16f acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
    // this wave's slices j = KS u + wave, in ascending order: slice j is the
    // (j % 4)-th 32-wide part of stage j / 4 (stage 2 u + wave / 4 for KS =
    // 8, chosen between two fixed arrays so that no pointer is indexed at
    // run time)
    const int js = wave & 3;
#pragma unroll
    for (int u = 0; u < DMA_K4_STAGES * 4 / KS; ++u) {
        const int j = KS * u + wave;
        const int s = j >> 2;
        if (s < nst && j < nsl) {
            const float *as = KS == 4 ? As[u] : ((wave >> 2) ? As[2 * u + 1] : As[2 * u]);
            const float *bs = KS == 4 ? Bs[u] : ((wave >> 2) ? Bs[2 * u + 1] : Bs[2 * u]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cc = 8 * js + 4 * h + q;  // chunk of this stage's 128 K
                f4 a = *(const f4 *)(as + l32 * 128 + 4 * (cc ^ (l32 & 15)));
                float b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int k = 32 * js + 16 * h + 4 * q + t;  // row of the Y block
                    b[t] = bs[k * 32 + 32 * (k >> 4) + l32];
                }
                if (!after) {
                    a = a * fx.a * fx.b;
#pragma unroll
                    for (int t = 0; t < 4; ++t) b[t] = b[t] * fy.a * fy.b;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[t], b[t], acc, 0, 0, 0);
            }
        }
    }

    // Every wave parks its partial tile in the first X blocks (wave w in
    // block w / 4); wave w then finishes register rows (16 / KS) w + i of the
    // tile: each element is the KS partial tiles added in wave order (the
    // order of one wave adding the others' into its own), scaled and stored,
    // its square added to the wave's sum; the waves' sums are then added in
    // wave order.  Spreading the epilogue over the waves instead of leaving
    // it to wave 0 shortens a small product's tail.
    constexpr int RPW = 16 / KS;  // register rows finished per wave
    double *wred = (double *)Bs[0];
    __syncthreads();
    {
        float *park = (wave >> 2) ? As[1] : As[0];
#pragma unroll
        for (int r = 0; r < 16; ++r) park[((wave & 3) * 16 + r) * 64 + lane] = acc[r];
    }
    __syncthreads();
    const PowScale fs = pow2_neg(after ? e.x + e.y : 0);
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int r = RPW * wave + i;
        float v = As[0][r * 64 + lane] + As[0][(16 + r) * 64 + lane];
#pragma unroll
        for (int g = 2; g < KS; ++g) v += As[g >> 2][((g & 3) * 16 + r) * 64 + lane];
        const int row = m0 + 8 * (r >> 2) + 4 * h + (r & 3);
        const int col = n0 + l32;
        if (row < n && col < n) {
            v = v * fs.a * fs.b;
            if constexpr (AXPI) v = fmaf(v, alpha, row == col ? 1.0f : 0.0f);
            C[(int64_t)row * n + col] = v;
            ss += (double)v * (double)v;
        }
    }
    ss = wave_sum_lane0(ss);
    if (lane == 0) wred[wave] = ss;
    __syncthreads();
    double t = 0.0;
    if (tid == 0) {
        t = wred[0];
#pragma unroll
        for (int w = 1; w < KS; ++w) t += wred[w];  // valid in thread 0
    }
    __syncthreads();  // the LDS blocks may be reused by the caller
    return t;
}

}  // namespace mpow
