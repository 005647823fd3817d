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
// Every output element is accumulated in the same order whatever BM, BN,
// WM, WN are (K tiles of 32 in ascending order, the same k-to-lane mapping),
// so all tile shapes give bit-identical products.
#pragma once

#include "scale_device.h"

namespace mpow {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int F32_BK = 32;          // K extent of one LDS tile
constexpr int F32_KH = F32_BK / 2;  // K values fed by each lane half
constexpr int F32_ALD = F32_BK + 4; // LDS row stride of the X tile (floats)

template <int BM, int BN>
struct F32TileLds {
    static constexpr int BLD = BN + 4;
    static constexpr int A_FLOATS = 2 * BM * F32_ALD;
    static constexpr int B_FLOATS = 2 * F32_BK * BLD;
};

// All threads of the workgroup (WM*WN waves) must call it.  `As` / `Bs` hold
// F32TileLds<BM,BN>::A_FLOATS / B_FLOATS floats of LDS, `red` WM*WN doubles.
// Returns the tile's sum of squares in thread 0 (0 elsewhere).
template <int BM, int BN, int WM, int WN, bool VEC>
__device__ __forceinline__ double f32_tile(const float *__restrict__ X, PowScale fx,
                                           const float *__restrict__ Y, PowScale fy,
                                           float *__restrict__ C, int n, int m0, int n0,
                                           float *As, float *Bs, double *red) {
    constexpr int NT = WM * WN * 64;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 32, FN = TN / 32;
    constexpr int BK = F32_BK, KH = F32_KH, ALD = F32_ALD;
    constexpr int BLD = F32TileLds<BM, BN>::BLD;
    constexpr int ABUF = BM * ALD, BBUF = BK * BLD;
    static_assert(FM >= 1 && FN >= 1 && TM % 32 == 0 && TN % 32 == 0, "wave tile");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, l32 = lane & 31;

    constexpr int AV = VEC ? 4 : 1;          // floats per load
    constexpr int LA = BM * BK / (AV * NT);  // loads per thread, X tile
    constexpr int LB = BK * BN / (AV * NT);  // loads per thread, Y tile
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
        float *as = As + buf * ABUF;
        float *bs = Bs + buf * BBUF;
        if constexpr (VEC) {
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
                a[st][i] = *(const f4 *)(as + (wm * TM + i * 32 + l32) * ALD + h * KH + 4 * q);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    b[st][t][j] = bs[(h * KH + 4 * q + t) * BLD + wn * TN + j * 32 + l32];
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

    // 32x32 accumulator layout: register r of lane l holds row
    // 8*(r/4) + 4*(l/32) + r%4 and column l%32 of the 32x32 block.
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
                    const float v = acc[i][j][r];
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
        for (int w = 0; w < WM * WN; ++w) t += red[w];
    }
    __syncthreads();  // red and the LDS tiles may be reused by the caller
    return t;
}

}  // namespace mpow
