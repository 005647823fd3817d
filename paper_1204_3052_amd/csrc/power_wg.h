// A whole power A^p of one matrix (n <= 256) computed by one workgroup of
// eight waves: the paper's repeated-squaring schedule (section 4.3) with its
// operands staged in the workgroup's local memory (sections 4.3.2, 4.3.6),
// every product held whole in the waves' accumulators.
//
// Why one workgroup and whole products: at these sizes a product is 2n^3
// flops (at most 34 MFLOP), a few microseconds of one CU's MFMA pipes, which
// is the cost of one dependent kernel launch.  One workgroup that keeps the
// running matrix next to its MFMA pipes pays no launch, no grid-wide wait
// and no per-tile prologue between products, and the per-step Frobenius
// norm is a reduction over its own accumulators.
//
//  - The product C = X Y is cut into 32 x 32 blocks (nb = ceil(n / 32) per
//    side); wave w owns blocks w, w + 8, w + 16, ... in row-major block
//    order (at most 8 blocks, 128 accumulator registers per lane), so the
//    waves' shares differ by at most one block.  Each block is accumulated
//    with v_mfma_f32_32x32x2_f32 in the k order of the other float32 tiles
//    (K tiles of 32 ascending, lane half h taking k = 16h + 4q + t), so the
//    products carry the same bits as theirs.
//  - n <= 128 (resident): the normalised base 2^-eA A and the running matrix
//    X stay in LDS for the whole power (two 128 x 128 float arrays, 128 KB).
//    Element (r, c) sits at r * 128 + 4 ((c / 4) ^ g(r)) + c % 4 with
//    g(r) = (r % 16) ^ (8 * ((r / 16) % 2)): the left operand's 16-byte reads
//    (rows r0 .. r0 + 15 of one chunk) and the right operand's 4-byte reads
//    (rows k and k + 16, 32 columns each) are free of bank conflicts.  After
//    each product the waves reduce the sum of squares of C, derive
//    e = floor(log2 ||C||_F), and write C * 2^-e over X.
//  - 128 < n <= 256 (panel): the running matrix and 2^-eA A live in two
//    n_pad x n_pad float arrays in memory (n_pad = 32 nb, zero padded, the
//    workgroup's own scratch), and each product streams K panels of 32
//    (n_pad x 32 of X, 32 x n_pad of Y) into two LDS stages by LDS-DMA
//    buffer loads, the next panel loading while the current one feeds the
//    MFMAs.  Each element of X and Y is read once per product.  Layouts as
//    the LDS-DMA tiles: X panel chunk c of row r at c ^ ((r / 2) % 8), Y panel
//    rows with bit 4 of k set swapping their 32-float halves.
//  - Scaling: operands are always the normalised matrices, so a product's
//    sums are those of the other kernels with scaled operands (exact powers
//    of two); s follows s <- 2 (s + eX) for a square and s <- s + eX + eA for
//    a multiply, and the output is C_G * 2^-e_G with log2 scale s + e_G, or
//    C_G * 2^s rounded to float32 through float64.
#pragma once

#include "gemm_f32_dma.h"
#include "scale_device.h"

namespace mpow {

constexpr int WG_NT = 512;         // threads of the workgroup (8 waves)
constexpr int WG_NW = 8;
constexpr int WG_RES_MAX_N = 128;  // LDS-resident up to this n
constexpr int WG_MAX_N = 256;      // panel path up to this n
constexpr int WG_RES_LD = 128;     // LDS row stride of a resident matrix (floats)
constexpr int WG_STAGE = 2 * 256 * 32;  // floats of one panel stage (X panel, then Y panel)
static_assert(WG_STAGE == WG_RES_LD * WG_RES_LD, "a stage array holds one resident matrix");

// Row stride of the panel path's matrices in memory.
__host__ __device__ constexpr int wg_npad(int n) { return (n + 31) / 32 * 32; }

namespace wgdetail {

__device__ __forceinline__ int res_swz(int r) { return (r & 15) ^ (((r >> 4) & 1) << 3); }
__device__ __forceinline__ int res_idx(int r, int c) {
    return r * WG_RES_LD + 4 * ((c >> 2) ^ res_swz(r)) + (c & 3);
}

// Block j of this wave: row and column of the block grid.
struct Blocks {
    int cnt;
    int bi[8], bj[8];
};
__device__ __forceinline__ Blocks wave_blocks(int nb, int wave) {
    Blocks b;
    const int T = nb * nb;
    b.cnt = wave < T ? (T - wave + WG_NW - 1) / WG_NW : 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int t = wave + WG_NW * j;
        b.bi[j] = t / nb;
        b.bj[j] = t % nb;
    }
    return b;
}

// Sum of squares of the valid part (row, col < n) of this wave's blocks,
// reduced over the workgroup in a fixed order; every thread gets it.
template <int MB>
__device__ __forceinline__ double wg_block_sumsq(const v16f (&acc)[MB], const Blocks &b, int n,
                                                 double *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, l32 = lane & 31;
    double ss = 0.0;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (j < b.cnt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = b.bi[j] * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int col = b.bj[j] * 32 + l32;
                if (row < n && col < n) ss += (double)acc[j][r] * (double)acc[j][r];
            }
        }
    }
    ss = wave_sum_lane0(ss);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    double S = 0.0;
#pragma unroll
    for (int w = 0; w < WG_NW; ++w) S += red[w];
    return S;
}

// Writes this wave's blocks of the final C to out (n x n, row-major):
// C * 2^-e with *scale = s + e (scale non-null), else C * 2^s rounded to
// float32 through float64.
template <int MB>
__device__ __forceinline__ void wg_write_out(const v16f (&acc)[MB], const Blocks &b, int n,
                                             float *out, double *scale, double S, int e, double s) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, l32 = lane & 31;
    const PowScale f = pow2_neg(e);
    double sc = s;
    sc = sc > 4000.0 ? 4000.0 : (sc < -4000.0 ? -4000.0 : sc);
    const int si = (int)sc;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        if (j < b.cnt) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = b.bi[j] * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                const int col = b.bj[j] * 32 + l32;
                if (row < n && col < n) {
                    const float v = acc[j][r];
                    out[(int64_t)row * n + col] = scale ? v * f.a * f.b : (float)ldexp((double)v, si);
                }
            }
        }
    }
    if (scale && threadIdx.x == 0) *scale = (S == 0.0) ? 0.0 : s + (double)e;
}

// One product of the resident path: acc = X Y with X = left and Y = right,
// both resident n_pad x n_pad matrices (nb blocks per side).
template <int MB>
__device__ __forceinline__ void res_product(v16f (&acc)[MB], const Blocks &b, int nb,
                                            const float *left, const float *right) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
    for (int kt = 0; kt < nb; ++kt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f4 a[MB];
            float bv[MB][4];
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                if (j < b.cnt) {
                    const int row = b.bi[j] * 32 + l32;
                    a[j] = *(const f4 *)(left + row * WG_RES_LD +
                                         4 * ((8 * kt + 4 * h + q) ^ res_swz(row)));
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        bv[j][t] = right[res_idx(32 * kt + 16 * h + 4 * q + t, b.bj[j] * 32 + l32)];
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < b.cnt)
                        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j][t], bv[j][t], acc[j], 0,
                                                                      0, 0);
        }
    }
}

// One product of the panel path: acc = X Y with X, Y n_pad x n_pad float
// matrices in memory (row stride n_pad, zero padded), K panels streamed
// through L0 / L1.  Ends with a workgroup barrier after the last panel.
template <int MB>
__device__ __forceinline__ void panel_product(v16f (&acc)[MB], const Blocks &b, int npad,
                                              const float *X, const float *Y, float *L0,
                                              float *L1) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = lane >> 5, l32 = lane & 31;
    const int nb = npad / 32;
    const int bytes = npad * npad * 4;
    const __amdgpu_buffer_rsrc_t rX =
        __builtin_amdgcn_make_buffer_rsrc((void *)X, (short)0, bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rY =
        __builtin_amdgcn_make_buffer_rsrc((void *)Y, (short)0, bytes, 0x00020000);
    constexpr unsigned OUT = 0x80000000u;  // beyond the buffer: reads zeros

    // K panel kt into stage st: X panel rows 8i .. 8i + 7 per 1 KB load
    // (i = wave, wave + 8, ...), Y panel row k per 1 KB load (k = wave + 8m).
    const int xrow = lane >> 3;          // row within a 1 KB X load
    const int xpos = lane & 7;           // chunk position within the row
    auto load_panel = [&](int kt, float *st) {
        for (int i = wave; i < npad / 8; i += WG_NW) {
            const int row = 8 * i + xrow;
            const int c = xpos ^ ((row >> 1) & 7);
            const unsigned off = (unsigned)((row * npad + 32 * kt + 4 * c) * 4);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rX, (lds_void_t *)(st + i * 256), 16, off, 0,
                                                     0, 0);
        }
        float *ys = st + 256 * 32;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int k = wave + WG_NW * m;
            const int col = (4 * lane) ^ (32 * ((k >> 4) & 1));
            const unsigned off =
                col < npad ? (unsigned)(((32 * kt + k) * npad + col) * 4) : OUT;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rY, (lds_void_t *)(ys + k * 256), 16, off, 0,
                                                     0, 0);
        }
    };

#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;

    auto body = [&](int kt, const float *st, float *nx) {
        if (kt + 1 < nb) load_panel(kt + 1, nx);
        const float *ys = st + 256 * 32;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            f4 a[MB];
            float bv[MB][4];
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                if (j < b.cnt) {
                    const int row = b.bi[j] * 32 + l32;
                    a[j] = *(const f4 *)(st + row * 32 + 4 * ((4 * h + q) ^ ((row >> 1) & 7)));
                    const int col = (b.bj[j] * 32 + l32) ^ (32 * h);
#pragma unroll
                    for (int t = 0; t < 4; ++t) bv[j][t] = ys[(16 * h + 4 * q + t) * 256 + col];
                }
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    if (j < b.cnt)
                        acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j][t], bv[j][t], acc[j], 0,
                                                                      0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the next panel is in LDS
        __syncthreads();
    };
    load_panel(0, L0);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    for (int kt = 0; kt < nb; kt += 2) {
        body(kt, L0, L1);
        if (kt + 1 < nb) body(kt + 1, L1, L0);
    }
}

}  // namespace wgdetail

// Sum of squares (float64) of an n x n matrix by the workgroup, fixed order;
// every thread gets it.  Contains barriers.
__device__ __forceinline__ double wg_matrix_sumsq(const float *__restrict__ M, int n, double *red) {
    const int64_t total = (int64_t)n * n;
    double acc = 0.0;
    constexpr int U = 8;
    for (int64_t b = threadIdx.x; b < total; b += WG_NT * U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = b + (int64_t)u * WG_NT;
            v[u] = i < total ? M[i] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc += (double)v[u] * (double)v[u];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
#pragma unroll
    for (int s = WG_NT / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double S = red[0];
    __syncthreads();
    return S;
}

// A^p of one n x n matrix (1 <= n <= WG_MAX_N, or <= WG_RES_MAX_N when
// RESIDENT_ONLY) by the calling workgroup of WG_NT threads, all of which
// must call it.  LDS: L0 and L1 (WG_STAGE floats each; two distinct arrays,
// so the compiler sees that loads into one do not alias reads from the
// other) and `red` (WG_NT doubles).  `scratch` (panel path only,
// n > WG_RES_MAX_N) holds 2 * wg_npad(n)^2 floats of this workgroup's own
// memory.  out may be A.  Contains barriers; returns with the workgroup
// synchronised.
template <bool RESIDENT_ONLY>
__device__ void wg_power(const float *A, int n, int64_t p, float *out, double *scale,
                         float *scratch, float *L0, float *L1, double *red) {
    using namespace wgdetail;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t total = (int64_t)n * n;

    if (p == 0) {
        for (int64_t i = tid; i < total; i += WG_NT) {
            const int64_t r = i / n, c = i - r * n;
            out[i] = (r == c) ? 1.0f : 0.0f;
        }
        if (scale && tid == 0) *scale = 0.0;
        __syncthreads();
        return;
    }
    const double SA = wg_matrix_sumsq(A, n, red);
    const int eA = exponent_of_sumsq(SA);
    if (p == 1) {
        // out = A (unscaled) or A * 2^-eA with scale eA; each element is read
        // and written by the same thread, so out may be A
        const PowScale f = pow2_neg(eA);
        for (int64_t i = tid; i < total; i += WG_NT) out[i] = scale ? A[i] * f.a * f.b : A[i];
        if (scale && tid == 0) *scale = (SA == 0.0) ? 0.0 : (double)eA;
        __syncthreads();
        return;
    }

    const int npad = wg_npad(n), nb = npad / 32;
    const bool resident = RESIDENT_ONLY || n <= WG_RES_MAX_N;
    const Blocks b = wave_blocks(nb, wave);
    const PowScale fa = pow2_neg(eA);
    // the normalised base: resident in L1 (as a 128-stride swizzled matrix)
    // or in scratch (stride npad); zero padded to npad in both
    float *SX = scratch, *SAm = scratch + (size_t)npad * npad;
    if (resident) {
        for (int i = tid; i < npad * npad; i += WG_NT) {
            const int r = i / npad, c = i - r * npad;
            L1[res_idx(r, c)] = (r < n && c < n) ? A[(int64_t)r * n + c] * fa.a * fa.b : 0.f;
        }
    } else {
        for (int i = tid; i < npad * npad; i += WG_NT) {
            const int r = i / npad, c = i - r * npad;
            SAm[i] = (r < n && c < n) ? A[(int64_t)r * n + c] * fa.a * fa.b : 0.f;
        }
        __builtin_amdgcn_s_waitcnt(0x0f70);
    }
    __syncthreads();

    const int top = 63 - __clzll((unsigned long long)p);
    int eX = eA;
    double s = 0.0;
    bool first = true;
    // RES: the resident path (at most 16 blocks, 2 per wave), else the panel
    // path (at most 64 blocks, 8 per wave)
    auto run = [&](auto res_tag) {
        constexpr bool RES = decltype(res_tag)::value;
        constexpr int MB = RES ? 2 : 8;
        v16f acc[MB];
        double S = 0.0;
        for (int bit = top - 1; bit >= 0; --bit) {
            for (int pass = 0; pass < 2; ++pass) {
                const bool mul = pass == 1;
                if (mul && !((p >> bit) & 1)) break;
                const bool last = bit == 0 && (mul || !(p & 1));
                if constexpr (RES) {
                    const float *left = first ? L1 : L0;
                    res_product<MB>(acc, b, nb, left, mul ? L1 : left);
                } else {
                    const float *left = first ? SAm : SX;
                    panel_product<MB>(acc, b, npad, left, mul ? SAm : left, L0, L1);
                }
                first = false;
                S = wg_block_sumsq<MB>(acc, b, n, red);  // barrier: X fully read
                s = mul ? s + (double)eX + (double)eA : 2.0 * (s + (double)eX);
                eX = exponent_of_sumsq(S);
                if (last) break;
                // C * 2^-e over the running matrix (its padding stays zero)
                const PowScale f = pow2_neg(eX);
                const int lane = tid & 63, h = lane >> 5, l32 = lane & 31;
#pragma unroll
                for (int j = 0; j < MB; ++j) {
                    if (j < b.cnt) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int row = b.bi[j] * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                            const int col = b.bj[j] * 32 + l32;
                            const float v = acc[j][r] * f.a * f.b;
                            if constexpr (RES)
                                L0[res_idx(row, col)] = v;
                            else
                                SX[row * npad + col] = v;
                        }
                    }
                }
                if constexpr (!RES) __builtin_amdgcn_s_waitcnt(0x0f70);  // stores done
                __syncthreads();
            }
        }
        wg_write_out<MB>(acc, b, n, out, scale, S, eX, s);
    };
    if (resident)
        run(DmaBool<true>{});
    else if constexpr (!RESIDENT_ONLY)
        run(DmaBool<false>{});
    __syncthreads();  // LDS and `red` may be reused by the caller
}

}  // namespace mpow
