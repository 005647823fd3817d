// One BM x BN output tile of the float32 product C = (2^-eX X)(2^-eY Y),
// computed by one workgroup (the paper's tiled product, section 4.3.7, with
// LDS tiles kept consistent by barriers, section 4.3.6).
//
// CDNA4 design:
//  - v_mfma_f32_32x32x2_f32 does the multiply-adds: each 64-lane wave owns a
//    (32*FM) x (32*FN) block of C in FM*FN accumulator tiles of 16 floats/lane.
//  - The K dimension of a 32-wide LDS tile is split between the two lane
//    halves: lanes 0-31 feed k in [0,16) and lanes 32-63 feed k in [16,32), so
//    a lane's A values for four successive MFMAs are contiguous in a row of
//    the A tile and come from one 16-byte LDS read.
//  - Tiles of X (BM x 32) and Y (32 x BN) are loaded from memory with
//    coalesced 16-byte loads (4-byte loads when n % 4 != 0), scaled by the
//    exact power of two 2^-e on the way, and stored to one of two LDS buffers
//    while the other one feeds the MFMAs.
//  - The epilogue stores C and returns the tile's float64 sum of squares
//    (fixed reduction order).
//
//  - K split (KS > 1, for small n where output tiles alone cannot fill the
//    chip): KS groups of WM x WN waves share the output tile; the LDS tile is
//    32*KS wide in K and group g takes its g-th 32-wide slice, so each group
//    sums every KS-th slice of K.  The epilogue adds the KS partial tiles in
//    group order 0, 1, ..., KS-1.
//
// With KS = 1 every output element is accumulated in the same order whatever
// BM, BN, WM, WN are (K tiles of 32 in ascending order, the same k-to-lane
// mapping), so those tile shapes give bit-identical products.  A K-split
// shape adds in another (fixed) order: deterministic, not bit-identical to
// the KS = 1 shapes.
#pragma once

#include "scale_device.h"

namespace mpow {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int F32_BK = 32;          // K extent of one LDS tile
constexpr int F32_KH = F32_BK / 2;  // K values fed by each lane half
constexpr int F32_ALD = F32_BK + 4; // LDS row stride of the X tile (floats)

template <int BM, int BN, int KS = 1>
struct F32TileLds {
    static constexpr int BKC = F32_BK * KS;  // K extent of one LDS tile
    static constexpr int ALD = BKC + 4;      // LDS row stride of the X tile
    static constexpr int BLD = BN + 4;       // LDS row stride of the Y tile
    static constexpr int A_FLOATS = 2 * BM * ALD;
    static constexpr int B_FLOATS = 2 * BKC * BLD;
};

// Operand scales 2^-eX and 2^-eY, returned by the caller's scale function.
struct OperandScales {
    PowScale x, y;
};

// All threads of the workgroup (WM*WN*KS waves) must call it.  `As` / `Bs`
// hold F32TileLds<BM,BN,KS>::A_FLOATS / B_FLOATS floats of LDS, `red`
// WM*WN doubles.
// `scales()` is called by every thread once, after the first tile's global
// loads are issued (so work it does, such as reducing partial sums, overlaps
// their latency); it may contain barriers.  Returns the tile's sum of squares
// in thread 0 (0 elsewhere).
//
// VEC selects the global loads: 0 = 4-byte loads (any n and alignment),
// 1 = 16-byte loads (n % 4 == 0, X and Y 16-byte aligned), 2 = chosen at run
// time by `vec` with the register footprint of 1 (for kernels that handle
// both cases and must not carry two copies of the tile loop).
//
// AXPI selects the epilogue C = alpha * (X'Y') + I (one fused multiply-add
// per element, the identity added on the diagonal) instead of C = X'Y'.
template <int BM, int BN, int WM, int WN, int VEC, int KS = 1, bool AXPI = false, typename ScaleFn>
__device__ __forceinline__ double f32_tile(const float *__restrict__ X, const float *__restrict__ Y,
                                           ScaleFn scales, float *__restrict__ C, int n, int m0,
                                           int n0, float *As, float *Bs, double *red,
                                           bool vec = VEC == 1, float alpha = 1.0f) {
    typedef F32TileLds<BM, BN, KS> L;
    constexpr int NT = WM * WN * KS * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;
    constexpr int BK = L::BKC, KH = F32_KH, ALD = L::ALD, BLD = L::BLD;
    constexpr int ABUF = BM * ALD, BBUF = BK * BLD;
    static_assert(FM >= 1 && FN >= 1 && TM % 32 == 0 && TN % 32 == 0, "wave tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int ks = wave / (WM * WN);          // K-split group
    const int wmn = wave % (WM * WN);
    const int wm = wmn / WN, wn = wmn % WN;
    const int h = lane >> 5, l32 = lane & 31;
    const int kg = ks * F32_BK;  // this group's K slice within an LDS tile

    constexpr bool V4 = VEC != 0;            // vector register layout
    constexpr int AV = V4 ? 4 : 1;           // floats per load slot
    constexpr int LA = BM * BK / (AV * NT);  // load slots per thread, X tile
    constexpr int LB = BK * BN / (AV * NT);  // load slots per thread, Y tile
    static_assert(LA * AV * NT == BM * BK && LB * AV * NT == BK * BN, "load split");
    f4 ra[V4 ? LA : 1];
    f4 rb[V4 ? LB : 1];
    float sa[V4 ? 1 : LA];
    float sb[V4 ? 1 : LB];

    // Four consecutive elements of row gr starting at column gc, zero past n.
    auto load4 = [&](const float *__restrict__ M, int gr, int gc) -> f4 {
        f4 v = {0.f, 0.f, 0.f, 0.f};
        if (VEC == 1 || vec) {
            if (gr < n && gc < n) v = *(const f4 *)(M + (int64_t)gr * n + gc);
        } else if (gr < n) {
            const float *p = M + (int64_t)gr * n + gc;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (gc + t < n) v[t] = p[t];
        }
        return v;
    };

    auto gload = [&](int k0) {
        if constexpr (V4) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
                ra[r] = load4(X, m0 + row, k0 + c);
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
                rb[r] = load4(Y, k0 + row, n0 + c);
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

    PowScale fx, fy;
    auto sstore = [&](int buf) {
        float *as = As + buf * ABUF;
        float *bs = Bs + buf * BBUF;
        if constexpr (V4) {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
                *(f4 *)(&as[row * ALD + c]) = ra[r] * fx.a * fx.b;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
                *(f4 *)(&bs[row * BLD + c]) = rb[r] * fy.a * fy.b;
            }
        } else {
#pragma unroll
            for (int r = 0; r < LA; ++r) {
                const int idx = tid + r * NT;
                as[(idx / BK) * ALD + idx % BK] = sa[r] * fx.a * fx.b;
            }
#pragma unroll
            for (int r = 0; r < LB; ++r) {
                const int idx = tid + r * NT;
                bs[(idx / BN) * BLD + idx % BN] = sb[r] * fy.a * fy.b;
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
    {
        const OperandScales sc = scales();
        fx = sc.x;
        fy = sc.y;
    }
    sstore(0);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const float *as = As + cur * ABUF;
        const float *bs = Bs + cur * BBUF;
        // Operands of the next group of four k values are read from LDS while
        // the MFMAs of the current group run (register double buffering).
        f4 a[2][FM];
        float b[2][4][FN];
        auto lds_load = [&](int q, int st) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
                a[st][i] = *(const f4 *)(as + (wm * TM + i * 32 + l32) * ALD + kg + h * KH + 4 * q);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[st][t][j] = bs[(kg + h * KH + 4 * q + t) * BLD + wn * TN + j * 32 + l32];
        };
        lds_load(0, 0);
#pragma unroll
        for (int q = 0; q < KH / 4; ++q) {
            const int st = q & 1;
            if (q + 1 < KH / 4) lds_load(q + 1, st ^ 1);
            // keep the reads above ahead of this group's MFMAs
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[st][i][t], b[st][t][j],
                                                                        acc[i][j], 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    if constexpr (KS > 1) {
        // Groups 1..KS-1 park their accumulators in the (now idle) LDS tiles;
        // group 0 adds them in group order.  Layout: [group-1][i][j][r][lane
        // of the WM*WN waves], so every access is one float per lane.
        constexpr int PER = WM * WN * 64 * FM * FN * 16;
        static_assert((KS - 1) * PER <= 2 * ABUF, "K-split partials fit in the X tiles");
        auto slot = [&](int g, int i, int j, int r) -> float * {
            return As + (g - 1) * PER + ((i * FN + j) * 16 + r) * (WM * WN * 64) + wmn * 64 + lane;
        };
        if (ks > 0) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) *slot(ks, i, j, r) = acc[i][j][r];
        }
        __syncthreads();
        if (ks == 0) {
#pragma unroll
            for (int g = 1; g < KS; ++g)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
#pragma unroll
                        for (int r = 0; r < 16; ++r) acc[i][j][r] += *slot(g, i, j, r);
        }
    }

    // 32x32 accumulator layout: register r of lane l holds row
    // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the 32x32 block.
    if (ks == 0) {
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
                        float v = acc[i][j][r];
                        if constexpr (AXPI) v = fmaf(v, alpha, row == col ? 1.0f : 0.0f);
                        C[(int64_t)row * n + col] = v;
                        ss += (double)v * (double)v;
                    }
                }
        ss = wave_sum_lane0(ss);
        if (lane == 0) red[wmn] = ss;
    }
    __syncthreads();
    double t = 0.0;
    if (tid == 0) {
#pragma unroll
        for (int w = 0; w < WM * WN; ++w) t += red[w];
    }
    __syncthreads();  // red and the LDS tiles may be reused by the caller
    return t;
}

}  // namespace mpow
