// Device helpers for the power-of-two scaling of the running matrix.
//
// After every product the running matrix X is rescaled by 2^-e with
// e = floor(log2 ||X||_F).  The Frobenius norm comes from per-tile partial
// sums of squares (float64) that the producing kernel writes; every consumer
// block reduces the same partial array in the same fixed order, so all blocks
// of a launch derive the same e, and repeated runs give identical bits.
#pragma once

#include <hip/hip_runtime.h>

namespace mpow {

// floor(log2 sqrt(S)) for a sum of squares S; 0 when S is 0, NaN or Inf
// (no scaling is applied then).  With S = m * 2^q, m in [0.5, 1):
// floor(log2 S) = q - 1 and floor(log2 sqrt S) = floor((q - 1) / 2).
__device__ __forceinline__ int exponent_of_sumsq(double S) {
    if (!(S > 0.0) || !isfinite(S)) return 0;
    int q;
    (void)frexp(S, &q);
    const int t = q - 1;
    return t >= 0 ? t / 2 : -((1 - t) / 2);
}

// The multiplier 2^-e as two float factors, each a normal float for any e a
// float32 matrix can produce (|e| < 160), so x * f.lo * f.hi is exact
// whenever the result is a normal float.
struct PowScale {
    float a, b;
};
__device__ __forceinline__ PowScale pow2_neg(int e) {
    const int h = e / 2;
    PowScale f;
    f.a = ldexpf(1.0f, -h);
    f.b = ldexpf(1.0f, -(e - h));
    return f;
}

// Sum of `count` float64 partials in a fixed order, returned to every thread
// of the block.  `red` is LDS scratch of NT doubles.  Contains barriers: all
// threads of the block must call it.
template <int NT>
__device__ __forceinline__ double block_sum_partials(const double *__restrict__ part, int count,
                                                     double *red) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < count; i += NT) acc += part[i];
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

namespace detail {
// Value of lane l + 32 (lanes 0 .. 31; v_permlane32_swap), of lane l ^ 16
// (ds_swizzle, xor mode) and of lane l + N within the lane's row of 16
// (DPP row_shl; lanes past the row's end read 0), for a double as two
// 32-bit halves.  Every lane of the wave must be active.
__device__ __forceinline__ double lane_plus32(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_permlane32_swap(hi, hi, false, false)[1],
                            __builtin_amdgcn_permlane32_swap(lo, lo, false, false)[1]);
}
__device__ __forceinline__ double lane_xor16(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_ds_swizzle(hi, 0x401F),
                            __builtin_amdgcn_ds_swizzle(lo, 0x401F));
}
template <int N>
__device__ __forceinline__ double lane_row_plus(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x100 + N, 0xf, 0xf, true),
                            __builtin_amdgcn_update_dpp(0, lo, 0x100 + N, 0xf, 0xf, true));
}
}  // namespace detail

// Fixed-order reduction of one double per lane across a 64-lane wave; the
// result is valid in lane 0: the tree v_l += v_(l + d) for d = 32, 16, ...,
// 1, the additions of __shfl_down's tree, by register-to-register lane
// moves (permlane, swizzle and DPP) instead of LDS permutes, whose latency
// each of the six steps waited out.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum_lane0(double v) {
    v += detail::lane_plus32(v);
    v += detail::lane_xor16(v);
    v += detail::lane_row_plus<8>(v);
    v += detail::lane_row_plus<4>(v);
    v += detail::lane_row_plus<2>(v);
    v += detail::lane_row_plus<1>(v);
    return v;
}

// Sum of `count` float64 partials by one wave, in a fixed order (lane l adds
// partials l, l + 64, ... in turn, then the wave's fixed tree), returned to
// every lane.  No barrier: each wave that calls it gets the same value.
__device__ __forceinline__ double wave_sum_partials(const double *__restrict__ part, int count) {
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int i = lane; i < count; i += 64) acc += part[i];
    acc = wave_sum_lane0(acc);
    return __shfl(acc, 0, 64);
}

// Sum of `count` float64 partials in a fixed order, returned to every thread
// of the block: up to 1024 partials each wave sums them all itself
// (wave_sum_partials: at most 16 loads per lane and a six-step shuffle tree,
// no barrier), more by the block's tree (block_sum_partials, nine barriers
// at 512 threads).  The choice depends on count alone, so every block of a
// launch adds in the same order.  For the partials of a small product the
// block's tree of barriers was a large part of the time a workgroup spends
// before its first MFMA: chains of products at n <= 256 ran 10-12% faster
// without it.  All threads of the block must call it (it may contain
// barriers).
template <int NT>
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int count,
                                               double *red) {
    if (count <= 1024) return wave_sum_partials(part, count);
    return block_sum_partials<NT>(part, count, red);
}

// Tile order for a grid of tilesM x tilesN output tiles.  Workgroups are
// dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b % 8), and
// each XCD has its own L2.  The block index is first permuted so that every
// XCD gets one contiguous range of tiles, and that range is walked in bands
// of GROUP_M tile rows, column by column, so that the workgroups an XCD runs
// at the same time share rows of X and columns of Y in its L2.  With 32 CUs
// per XCD, the 32 concurrent tiles form a GROUP_M x (32 / GROUP_M) block,
// which reads GROUP_M row panels of X and 32 / GROUP_M column panels of Y:
// 8 suits square tiles, 4 tiles twice as tall as wide.  A bijection of
// [0, tilesM * tilesN).
template <int GROUP_M = 8>
__device__ __forceinline__ void tile_of_block(int b, int tilesM, int tilesN, int *tm, int *tn) {
    constexpr int XCDS = 8;
    const int T = tilesM * tilesN;
    int t = b;
    if (T >= 4 * XCDS) {
        const int x = b % XCDS, local = b / XCDS;
        const int base = T / XCDS, rem = T % XCDS;
        t = x * base + (x < rem ? x : rem) + local;
    }
    const int band = GROUP_M * tilesN;
    const int first_m = (t / band) * GROUP_M;
    const int gm = tilesM - first_m < GROUP_M ? tilesM - first_m : GROUP_M;
    const int r = t % band;
    *tm = first_m + r % gm;
    *tn = r / gm;
}

}  // namespace mpow
