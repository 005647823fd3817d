// A whole power A^p of one matrix (n <= 256) computed by one workgroup: the
// paper's repeated-squaring schedule (section 4.3) with its operands staged
// in the workgroup's local memory (sections 4.3.2, 4.3.6), every product
// held whole in the waves' accumulators.
//
// Why one workgroup and whole products: at these sizes a product is 2n^3
// flops (at most 34 MFLOP), a few microseconds of one CU's MFMA pipes, which
// is the cost of one dependent kernel launch.  One workgroup that keeps the
// running matrix next to its MFMA pipes pays no launch, no grid-wide wait
// and no per-tile prologue between products, and the per-step Frobenius
// norm is a reduction over its own accumulators.
//
//  - The product C = X Y is cut into 32 x 32 blocks (nb = ceil(n / 32) per
//    side), each accumulated by one wave with v_mfma_f32_32x32x2_f32 in the
//    k order of the other float32 tiles (K tiles of 32 ascending, lane half
//    h taking k = 16h + 4q + t), so the products carry the same bits as
//    theirs.
//  - Resident form (n <= LD, LD = 64 or 128): the normalised base 2^-eA A
//    and the running matrix X stay in LDS for the whole power (two LD x LD
//    float arrays: 32 KB for LD = 64, 128 KB for LD = 128).  Element (r, c)
//    sits at r * LD + 4 ((c / 4) ^ g(r)) + c % 4 with
//    g(r) = (r % 16) ^ (8 * ((r / 16) % 2)): the left operand's 16-byte
//    reads (rows r0 .. r0 + 15 of one chunk) and the right operand's 4-byte
//    reads (rows k and k + 16, 32 columns each) are free of bank conflicts.
//    Wave w owns blocks w, w + NW, ... in row-major block order.  After each
//    product the waves reduce the sum of squares of C, derive
//    e = floor(log2 ||C||_F), and write C * 2^-e over X.
//  - Panel form (n <= NPMAX): the running matrix and 2^-eA A live in two
//    n_pad x n_pad float arrays in memory (n_pad = 32 nb, zero padded, the
//    workgroup's own scratch), and each product streams K panels of 32
//    (n_pad x 32 of X, 32 x n_pad of Y) into two LDS stages by LDS-DMA
//    buffer loads, the next panel loading while the current one feeds the
//    MFMAs; each element of X and Y is read once per product.  Each of the
//    NW = 8 or 16 waves owns consecutive blocks of one block column, at
//    most ceil(nb^2 / NW) of them, and the waves that share a SIMD own the
//    balanced share ceil(nb^2 / 4) or less together (a fixed table per nb):
//    a wave reads each right-operand value once for all its blocks, and
//    every MFMA's operands are fixed at compile time.  For n <= 256 sixteen
//    waves hold at most four blocks each (64 accumulator registers), which
//    leaves registers to read the next step's operands while the MFMAs of
//    the current one run.
//    The number of blocks selects a fully unrolled instance of the K loop.
//    Layouts as the LDS-DMA tiles: X panel chunk c of row r at
//    c ^ ((r / 2) % 8), Y panel rows with bit 4 of k set swapping their
//    32-float halves.
//  - Scaling: the resident form's operands are always the normalised
//    matrices; the panel form keeps each product in memory as computed, with
//    its exponent, and scales the next product's sums by the operands'
//    exponents, as the product kernels do in their epilogue.  Either way a
//    product's sums are those of the other kernels (exact powers of two,
//    wherever nothing is subnormal); s follows s <- 2 (s + eX) for a square and s <- s + eX + eA for
//    a multiply, and the output is C_G * 2^-e_G with log2 scale s + e_G, or
//    C_G * 2^s rounded to float32 through float64.
#pragma once

#include "gemm_f32_dma.h"
#include "scale_device.h"

namespace mpow {

constexpr int WG_RES_MAX_N = 128;  // resident form up to this n
constexpr int WG_MAX_N = 256;      // panel form up to this n

// Row stride of the panel form's matrices in memory.
__host__ __device__ constexpr int wg_npad(int n) { return (n + 31) / 32 * 32; }

// LDS of the resident form: two LD x LD float arrays.
template <int LD>
struct WgResLds {
    static constexpr int FLOATS = LD * LD;
};
// LDS of the panel form: one stage holds an NPMAX x 32 X panel and a
// 32 x NPMAX Y panel; two stages alternate.
template <int NPMAX>
struct WgPanelLds {
    static constexpr int STAGE = 2 * NPMAX * 32;
};

namespace wgdetail {

__device__ __forceinline__ int res_swz(int r) { return (r & 15) ^ (((r >> 4) & 1) << 3); }
template <int LD>
__device__ __forceinline__ int res_idx(int r, int c) {
    return r * LD + 4 * ((c >> 2) ^ res_swz(r)) + (c & 3);
}

// Fixed-order workgroup sum of one double per thread (wave trees, then the
// waves in order); every thread gets it.  Contains a barrier; `red` holds NW
// doubles and must not be written again before the next barrier.
template <int NW>
__device__ __forceinline__ double wg_sum(double v, double *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum_lane0(v);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double S = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) S += red[w];
    return S;
}

// Sum of squares of the valid part (row, col < n) of one 32 x 32 block.
__device__ __forceinline__ double block_sumsq(const v16f &acc, int bi, int bj, int n) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int col = bj * 32 + l32;
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = bi * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (row < n && col < n) ss += (double)acc[r] * (double)acc[r];
    }
    return ss;
}

// Writes the valid part of one block of the final C to out (n x n,
// row-major): C * 2^-e (scaled) or C * 2^si rounded through float64.
__device__ __forceinline__ void block_write_out(const v16f &acc, int bi, int bj, int n, float *out,
                                                bool scaled, PowScale f, int si) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int col = bj * 32 + l32;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = bi * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
        if (row < n && col < n)
            out[(int64_t)row * n + col] =
                scaled ? acc[r] * f.a * f.b : (float)ldexp((double)acc[r], si);
    }
}

// Sum of squares (float64) of an n x n matrix in memory by the workgroup of
// NT threads, fixed order (16-byte loads when n % 4 == 0 and M is 16-byte
// aligned, eight in flight per thread); every thread gets it.  Contains
// barriers; `red` holds NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double matrix_sumsq(const float *__restrict__ M, int n, double *red) {
    const int64_t total = (int64_t)n * n;
    double acc = 0.0;
    constexpr int U = 8;
    if ((n & 3) == 0 && ((uintptr_t)M & 15) == 0) {
        const f4 *M4 = (const f4 *)M;
        const int64_t t4 = total / 4;
        for (int64_t b = threadIdx.x; b < t4; b += NT * U) {
            f4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                v[u] = i < t4 ? M4[i] : f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc += (double)v[u][c] * (double)v[u][c];
        }
    } else {
        for (int64_t b = threadIdx.x; b < total; b += NT * U) {
            float v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = b + (int64_t)u * NT;
                v[u] = i < total ? M[i] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += (double)v[u] * (double)v[u];
        }
    }
    const double S = wg_sum<NT / 64>(acc, red);
    __syncthreads();  // `red` is free again
    return S;
}

// The normalised base 2^-eA A, zero padded to npad x npad: store(r, c, v)
// receives four consecutive columns c .. c + 3 (c % 4 == 0) of row r.  With
// n % 4 == 0 and a 16-byte aligned A the input is read by 16-byte loads,
// four in flight per thread.
template <int NT, typename Store4>
__device__ __forceinline__ void copy_base_padded(const float *__restrict__ A, int n, int npad,
                                                 PowScale f, Store4 store) {
    const int q = npad / 4;
    const int total4 = npad * q;
    constexpr int U = 4;
    if ((n & 3) == 0 && ((uintptr_t)A & 15) == 0) {
        const f4 *A4 = (const f4 *)A;
        const int nq = n / 4;
        for (int b = threadIdx.x; b < total4; b += NT * U) {
            f4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = b + u * NT;
                const int r = i / q, c4 = i - r * q;
                v[u] = (i < total4 && r < n && c4 < nq) ? A4[r * nq + c4] * f.a * f.b
                                                          : f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = b + u * NT;
                if (i < total4) {
                    const int r = i / q;
                    store(r, 4 * (i - r * q), v[u]);
                }
            }
        }
    } else {
        for (int i = threadIdx.x; i < total4; i += NT) {
            const int r = i / q, c = 4 * (i - r * q);
            f4 v;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[k] = (r < n && c + k < n) ? A[(int64_t)r * n + c + k] * f.a * f.b : 0.f;
            store(r, c, v);
        }
    }
}

// The first steps shared by both forms: p = 0 (identity) and p = 1 (A, or
// A * 2^-eA with scale eA) are written out here and return false; otherwise
// *SA and *eA are the input's sum of squares and exponent.
template <int NT>
__device__ __forceinline__ bool power_head(const float *A, int n, int64_t p, float *out,
                                           double *scale, double *red, double *SA, int *eA) {
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)n * n;
    if (p == 0) {
        for (int64_t i = tid; i < total; i += NT) {
            const int64_t r = i / n, c = i - r * n;
            out[i] = (r == c) ? 1.0f : 0.0f;
        }
        if (scale && tid == 0) *scale = 0.0;
        __syncthreads();
        return false;
    }
    *SA = matrix_sumsq<NT>(A, n, red);
    *eA = exponent_of_sumsq(*SA);
    if (p == 1) {
        // each element is read and written by the same thread, so out may be A
        const PowScale f = pow2_neg(*eA);
        for (int64_t i = tid; i < total; i += NT) out[i] = scale ? A[i] * f.a * f.b : A[i];
        if (scale && tid == 0) *scale = (*SA == 0.0) ? 0.0 : (double)*eA;
        __syncthreads();
        return false;
    }
    return true;
}

// ------------------------------------------------------------ resident form

// One product of the resident form: acc = X Y with X = left, Y = right
// (resident, row stride LD, nb blocks per side); the wave owns CNT blocks,
// wave + NW j.
template <int LD, int NW, int CNT, int MB>
__device__ __forceinline__ void res_product(v16f (&acc)[MB], int nb, int wave, const float *left,
                                            const float *right) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, l32 = lane & 31;
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
    int bi[MB], bj[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        const int t = wave + NW * j;
        bi[j] = t / nb;
        bj[j] = t - bi[j] * nb;
    }
    // operands of K step (kt, q); the reads of the next step are issued
    // before the MFMAs of the current one, so their LDS latency is hidden
    struct Ops {
        f4 a[MB];
        float b[MB][4];
    };
    auto read = [&](Ops &o, int kt, int q) {
#pragma unroll
        for (int j = 0; j < CNT; ++j) {
            const int row = bi[j] * 32 + l32;
            o.a[j] = *(const f4 *)(left + row * LD + 4 * ((8 * kt + 4 * h + q) ^ res_swz(row)));
#pragma unroll
            for (int t = 0; t < 4; ++t)
                o.b[j][t] = right[res_idx<LD>(32 * kt + 16 * h + 4 * q + t, bj[j] * 32 + l32)];
        }
    };
    Ops ops[2];
    read(ops[0], 0, 0);
    for (int kt = 0; kt < nb; ++kt) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < 3)
                read(ops[(q + 1) & 1], kt, q + 1);
            else if (kt + 1 < nb)
                read(ops[0], kt + 1, 0);
            const Ops &o = ops[q & 1];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int j = 0; j < CNT; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a[j][t], o.b[j][t], acc[j], 0, 0, 0);
        }
    }
}

// The power's products for a wave with CNT blocks; see wg_power_resident.
template <int LD, int NW, int CNT, int MB>
__device__ __forceinline__ void res_power_body(int n, int64_t p, float *out, double *scale,
                                               float *LX, float *LA, double *red, int eA,
                                               int wave) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int nb = wg_npad(n) / 32;
    int bi[MB], bj[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) {
        const int t = wave + NW * j;
        bi[j] = t / nb;
        bj[j] = t - bi[j] * nb;
    }
    const int top = 63 - __clzll((unsigned long long)p);
    int eX = eA;
    double s = 0.0, S = 0.0;
    bool first = true;
    v16f acc[MB];
    for (int bit = top - 1; bit >= 0; --bit) {
        for (int pass = 0; pass < 2; ++pass) {
            const bool mul = pass == 1;
            if (mul && !((p >> bit) & 1)) break;
            const bool last = bit == 0 && (mul || !(p & 1));
            const float *left = first ? LA : LX;
            res_product<LD, NW, CNT, MB>(acc, nb, wave, left, mul ? LA : left);
            first = false;
            double ss = 0.0;
#pragma unroll
            for (int j = 0; j < CNT; ++j) ss += block_sumsq(acc[j], bi[j], bj[j], n);
            S = wg_sum<NW>(ss, red);  // barrier: X fully read
            s = mul ? s + (double)eX + (double)eA : 2.0 * (s + (double)eX);
            eX = exponent_of_sumsq(S);
            if (last) break;
            // C * 2^-e over the running matrix; its padding is written as
            // zeros (a non-finite operand value makes the padding of C NaN,
            // 0 * inf, which must not reach the next product's sums)
            const PowScale f = pow2_neg(eX);
#pragma unroll
            for (int j = 0; j < CNT; ++j) {
                const int col = bj[j] * 32 + l32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = bi[j] * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
                    LX[res_idx<LD>(row, col)] = (row < n && col < n) ? acc[j][r] * f.a * f.b : 0.0f;
                }
            }
            __syncthreads();
        }
    }
    double sc = s;
    sc = sc > 4000.0 ? 4000.0 : (sc < -4000.0 ? -4000.0 : sc);
    const PowScale f = pow2_neg(eX);
#pragma unroll
    for (int j = 0; j < CNT; ++j)
        block_write_out(acc[j], bi[j], bj[j], n, out, scale != nullptr, f, (int)sc);
    if (scale && threadIdx.x == 0) *scale = (S == 0.0) ? 0.0 : s + (double)eX;
}

}  // namespace wgdetail

// A^p of one n x n matrix, 1 <= n <= LD, by the calling workgroup of NW
// waves (all of which must call it), base and running matrix resident in
// LDS: LX and LA hold LD * LD floats each, `red` NW doubles.  out may be A.  Contains barriers; returns with the workgroup synchronised.
template <int LD, int NW>
__device__ __forceinline__ void wg_power_resident(const float *A, int n, int64_t p, float *out, double *scale,
                                  float *LX, float *LA, double *red) {
    using namespace wgdetail;
    constexpr int NT = NW * 64;
    constexpr int MB = ((LD / 32) * (LD / 32) + NW - 1) / NW;
    static_assert(MB >= 1 && MB <= 2, "resident forms hold at most two blocks per wave");
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double SA;
    int eA;
    if (!power_head<NT>(A, n, p, out, scale, red, &SA, &eA)) return;

    const int npad = wg_npad(n), nb = npad / 32;
    const PowScale fa = pow2_neg(eA);
    // the normalised base, zero padded to npad (a 4-column group of a row is
    // one 16-byte chunk of the swizzled layout)
    copy_base_padded<NT>(A, n, npad, fa, [&](int r, int c, f4 v) {
        *(f4 *)(LA + res_idx<LD>(r, c)) = v;
    });
    __syncthreads();

    const int T = nb * nb;
    const int cnt = wave < T ? (T - wave + NW - 1) / NW : 0;
    // every wave takes part in the barriers of every product, whatever its count
    switch (cnt) {
        case 0: res_power_body<LD, NW, 0, MB>(n, p, out, scale, LX, LA, red, eA, wave); break;
        case 1: res_power_body<LD, NW, 1, MB>(n, p, out, scale, LX, LA, red, eA, wave); break;
        default:
            if constexpr (MB >= 2) res_power_body<LD, NW, 2, MB>(n, p, out, scale, LX, LA, red, eA, wave);
            break;
    }
    __syncthreads();  // LDS and `red` may be reused by the caller
}

// --------------------------------------------------------------- panel form

namespace wgdetail {

// Which blocks each wave of the panel form owns, for nb = npad / 32 blocks
// per side: entry [nb - 1][w] = c | r0 << 4 | cnt << 8 gives wave w block
// rows r0 .. r0 + cnt - 1 of block column c.  Every wave's blocks lie in one
// block column (its right-operand values serve all of them, and no MFMA
// has to choose between two columns), no wave holds more than
// ceil(nb^2 / NW) blocks, and the waves of each SIMD (w, w + 4, ...) hold
// at most ceil(nb^2 / 4) blocks together, the balanced share; pieces_ok
// checks all of this at compile time.  (A column cut into ceil(nb / m)
// near-equal pieces of at most m = ceil(nb^2 / NW) blocks gives at most NW
// pieces here; they were placed on the SIMDs by exhaustive search.)
constexpr unsigned short kPieces16[8][16] = {
    {0x100, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000},  // nb = 1
    {0x100, 0x110, 0x101, 0x111, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000},  // nb = 2
    {0x100, 0x101, 0x102, 0x000, 0x110, 0x111, 0x112, 0x000, 0x120, 0x121, 0x122, 0x000, 0x000, 0x000, 0x000, 0x000},  // nb = 3
    {0x100, 0x101, 0x102, 0x103, 0x110, 0x111, 0x112, 0x113, 0x120, 0x121, 0x122, 0x123, 0x130, 0x131, 0x132, 0x133},  // nb = 4
    {0x200, 0x221, 0x203, 0x224, 0x220, 0x202, 0x223, 0x143, 0x201, 0x222, 0x204, 0x144, 0x140, 0x141, 0x142, 0x000},  // nb = 5
    {0x300, 0x331, 0x303, 0x334, 0x330, 0x302, 0x333, 0x305, 0x301, 0x332, 0x304, 0x335, 0x000, 0x000, 0x000, 0x000},  // nb = 6
    {0x400, 0x403, 0x406, 0x343, 0x401, 0x404, 0x340, 0x344, 0x402, 0x405, 0x341, 0x345, 0x000, 0x000, 0x342, 0x346},  // nb = 7
    {0x400, 0x402, 0x404, 0x406, 0x440, 0x442, 0x444, 0x446, 0x401, 0x403, 0x405, 0x407, 0x441, 0x443, 0x445, 0x447},  // nb = 8
};
constexpr unsigned short kPieces8[4][8] = {
    {0x100, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000, 0x000},  // nb = 1
    {0x100, 0x110, 0x101, 0x111, 0x000, 0x000, 0x000, 0x000},  // nb = 2
    {0x200, 0x201, 0x202, 0x000, 0x120, 0x121, 0x122, 0x000},  // nb = 3
    {0x200, 0x201, 0x202, 0x203, 0x220, 0x221, 0x222, 0x223},  // nb = 4
};

template <int NW, int NBMAX>
constexpr bool pieces_ok(const unsigned short (&t)[NBMAX][NW]) {
    for (int nb = 1; nb <= NBMAX; ++nb) {
        int cover[16][16] = {};
        int simd[4] = {};
        const int m = (nb * nb + NW - 1) / NW, share = (nb * nb + 3) / 4;
        for (int w = 0; w < NW; ++w) {
            const int c = t[nb - 1][w] & 15, r0 = (t[nb - 1][w] >> 4) & 15, cnt = t[nb - 1][w] >> 8;
            if (cnt > m || (cnt > 0 && (c >= nb || r0 + cnt > nb))) return false;
            for (int r = r0; r < r0 + cnt; ++r) cover[r][c] += 1;
            simd[w % 4] += cnt;
        }
        for (int i = 0; i < 4; ++i)
            if (simd[i] > share) return false;
        for (int r = 0; r < nb; ++r)
            for (int c = 0; c < nb; ++c)
                if (cover[r][c] != 1) return false;
    }
    return true;
}
static_assert(pieces_ok<16, 8>(kPieces16) && pieces_ok<8, 4>(kPieces8),
              "every block owned once, by waves of balanced SIMDs");

// K panel kt of X and Y (npad x npad in memory, row stride npad) into stage
// `st` by LDS-DMA: X panel rows 8i .. 8i + 7 per 1 KB load, Y panel rows
// 256 / YW per 1 KB load (YW = NPMAX floats per Y row); Y columns at or past
// npad read zeros.
template <int NPMAX, int NW>
__device__ __forceinline__ void panel_load(__amdgpu_buffer_rsrc_t rX, __amdgpu_buffer_rsrc_t rY,
                                           int npad, int kt, float *st, int wave) {
    constexpr int YW = NPMAX;
    constexpr int RPL = 256 / YW;  // Y rows per load
    constexpr int LPR = YW / 4;    // lanes per Y row
    constexpr unsigned OUT = 0x80000000u;
    // The lane's offsets are recomputed at every call (a few VALU
    // instructions) rather than kept across the product's K loop: the empty
    // asm hides the thread index's origin from loop-invariant hoisting.
    // Kept live, they were spilled, and the reload before a load waited for
    // every load in flight, the previous X panel's included (vmcnt(0)).
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int xrow = lane >> 3, xpos = lane & 7;
    for (int i = wave; i < npad / 8; i += NW) {
        const int row = 8 * i + xrow;
        const int c = xpos ^ ((row >> 1) & 7);
        const unsigned off = (unsigned)((row * npad + 32 * kt + 4 * c) * 4);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rX, (lds_void_t *)(st + i * 256), 16, off, 0, 0, 0);
    }
    float *ys = st + NPMAX * 32;
#pragma unroll
    for (int m = wave; m < 32 / RPL; m += NW) {
        const int k = m * RPL + lane / LPR;
        const int col = (4 * (lane % LPR)) ^ (32 * ((k >> 4) & 1));
        const unsigned off = col < npad ? (unsigned)(((32 * kt + k) * npad + col) * 4) : OUT;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rY, (lds_void_t *)(ys + m * 256), 16, off, 0, 0, 0);
    }
}

// Operands of one q step of a K panel: the left operand's 16-byte reads of
// the wave's CNT blocks and the right operand's four values of their block
// column.
template <int CNT>
struct PanelOps {
    f4 a[CNT > 0 ? CNT : 1];
    float b[4];
};

template <int NPMAX, int CNT, int MB>
__device__ __forceinline__ void panel_ops(PanelOps<CNT> &o, const float *st, const int (&bi)[MB],
                                          int col, int q) {
    constexpr int YW = NPMAX;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, l32 = lane & 31;
    const float *ys = st + NPMAX * 32;
#pragma unroll
    for (int t = 0; t < 4; ++t) o.b[t] = ys[(16 * h + 4 * q + t) * YW + col];
#pragma unroll
    for (int j = 0; j < CNT; ++j) {
        const int row = bi[j] * 32 + l32;
        o.a[j] = *(const f4 *)(st + row * 32 + 4 * ((4 * h + q) ^ ((row >> 1) & 7)));
    }
}

// The MFMAs of one K panel for a wave that owns CNT blocks of block column
// c0 (block rows bi[j]).  The q steps are unrolled over two operand sets, so
// the reads of step q + 1 are in flight while the MFMAs of step q run.
template <int NPMAX, int CNT, int MB>
__device__ __forceinline__ void panel_mfma(v16f (&acc)[MB], const float *st, const int (&bi)[MB],
                                           int c0) {
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, l32 = lane & 31;
    const int col = (c0 * 32 + l32) ^ (32 * h);
    PanelOps<CNT> ops[2];
    panel_ops<NPMAX, CNT, MB>(ops[0], st, bi, col, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < 3) panel_ops<NPMAX, CNT, MB>(ops[(q + 1) & 1], st, bi, col, q + 1);
        const PanelOps<CNT> &o = ops[q & 1];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < CNT; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(o.a[j][t], o.b[t], acc[j], 0, 0, 0);
    }
}

// One product of the panel form, acc = X Y (X, Y npad x npad in memory,
// zero padded), for a wave with CNT blocks.  Ends with a workgroup barrier
// after the last panel.
template <int NPMAX, int NW, int CNT, int MB>
__device__ __forceinline__ void panel_product(v16f (&acc)[MB], const int (&bi)[MB], int c0,
                                              int npad, const float *X, const float *Y, float *L0,
                                              float *L1, int wave) {
    const int nb = npad / 32;
    const int bytes = npad * npad * 4;
    const __amdgpu_buffer_rsrc_t rX =
        __builtin_amdgcn_make_buffer_rsrc((void *)X, (short)0, bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t rY =
        __builtin_amdgcn_make_buffer_rsrc((void *)Y, (short)0, bytes, 0x00020000);
#pragma unroll
    for (int j = 0; j < MB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
    panel_load<NPMAX, NW>(rX, rY, npad, 0, L0, wave);
    __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): the panel is in LDS
    __syncthreads();
    for (int kt = 0; kt < nb; kt += 2) {
        if (kt + 1 < nb) panel_load<NPMAX, NW>(rX, rY, npad, kt + 1, L1, wave);
        panel_mfma<NPMAX, CNT, MB>(acc, L0, bi, c0);
        __builtin_amdgcn_s_waitcnt(0x0f70);
        __syncthreads();
        if (kt + 1 < nb) {
            if (kt + 2 < nb) panel_load<NPMAX, NW>(rX, rY, npad, kt + 2, L0, wave);
            panel_mfma<NPMAX, CNT, MB>(acc, L1, bi, c0);
            __builtin_amdgcn_s_waitcnt(0x0f70);
            __syncthreads();
        }
    }
}

// Sum of squares (float64) of all 32 x 32 values of one block of the panel
// form, in the register order of block_sumsq.  The padding needs no mask: it
// is exactly zero while every operand value is finite (the operands' padding
// is stored as zeros), so adding its squares changes no partial sum; and a
// non-finite value there comes from a non-finite operand value, which makes
// the sum over the valid part non-finite as well (exponent 0 either way).
__device__ __forceinline__ double block_sumsq_all(const v16f &acc) {
    double ss = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) ss += (double)acc[r] * (double)acc[r];
    return ss;
}

// A product stays in memory as computed (its power-of-two scale applied to
// the next product's sums) while its exponent is at least this, so that the
// next product's two operand exponents add up to at least -32: the range in
// which the product kernels also scale in their epilogue.
constexpr int kPanelRawMinExp = -16;

// The power's products for a wave with CNT blocks, block rows r0 .. r0 +
// CNT - 1 of block column c0 (CNT fixed, so the K loop is fully unrolled
// over the blocks); see wg_power_panel.
//
// The running matrix in memory is N * 2^t, N the normalised matrix (norm in
// [1, 2)) and t its stored exponent.  A product of stored operands with
// exponents tl and tr gives the sums of the normalised product times
// 2^(tl + tr), exactly (power-of-two scaling commutes with every rounding
// while nothing is subnormal); they are scaled by 2^-(tl + tr) before use.
// The result C (norm below 4) is written back as it is, t = e(C), before its
// exponent is known, so the stores drain while the waves sum its squares,
// and one barrier covers both.  Only where e(C) < kPanelRawMinExp (a
// product far below norm 1) is it rewritten as C * 2^-e with t = 0.
template <int NPMAX, int NW, int CNT, int MB>
__device__ __forceinline__ void panel_power_body(const float *A, int n, int64_t p, float *out,
                                                 double *scale, float *SX, float *SAm, float *L0,
                                                 float *L1, double *red, int eA, int c0, int r0,
                                                 int wave) {
    const int lane = threadIdx.x & 63, h = lane >> 5, l32 = lane & 31;
    const int npad = wg_npad(n);
    int bi[MB];
#pragma unroll
    for (int j = 0; j < MB; ++j) bi[j] = r0 + j;

    const int top = 63 - __clzll((unsigned long long)p);
    int eX = eA;
    int tX = 0;  // stored exponent of the running matrix in SX
    double s = 0.0, S = 0.0;
    bool first = true;
    v16f acc[MB];
    const __amdgpu_buffer_rsrc_t rS =
        __builtin_amdgcn_make_buffer_rsrc((void *)SX, (short)0, npad * npad * 4, 0x00020000);
    // stores C * f of the wave's blocks into SX: buffer stores with one
    // offset register per block and the row offsets in scalar registers
    auto store_blocks = [&](float fa, float fb) {
#pragma unroll
        for (int j = 0; j < CNT; ++j) {
            const int vo = ((bi[j] * 32 + 4 * h) * npad + c0 * 32 + l32) * 4;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int so = (8 * (r >> 2) + (r & 3)) * npad * 4;
                __builtin_amdgcn_raw_buffer_store_b32(
                    __builtin_bit_cast(unsigned, acc[j][r] * fa * fb), rS, vo, so, 0);
            }
        }
    };
    // zeros over the padding of the wave's blocks on the matrix's edge: a
    // non-finite operand value makes it NaN (0 * inf), which must not reach
    // the next product's sums (elsewhere it is exactly zero already)
    auto zero_padding = [&]() {
#pragma unroll
        for (int j = 0; j < CNT; ++j) {
            if ((bi[j] + 1) * 32 <= n && (c0 + 1) * 32 <= n) continue;
            const int lim = c0 * 32 + l32 < n ? n - bi[j] * 32 - 4 * h : 0;  // rows below lim are valid
#pragma unroll
            for (int r = 0; r < 16; ++r)
                if (8 * (r >> 2) + (r & 3) >= lim) acc[j][r] = 0.0f;
        }
    };
    for (int bit = top - 1; bit >= 0; --bit) {
        for (int pass = 0; pass < 2; ++pass) {
            const bool mul = pass == 1;
            if (mul && !((p >> bit) & 1)) break;
            const bool last = bit == 0 && (mul || !(p & 1));
            const float *left = first ? SAm : SX;
            const int tl = first ? 0 : tX, tr = mul ? 0 : tl;
            panel_product<NPMAX, NW, CNT, MB>(acc, bi, c0, npad, left, mul ? SAm : left, L0, L1,
                                              wave);
            first = false;
            // (ends with a barrier: SX is no longer read)
            if (tl + tr != 0) {
                const PowScale fs = pow2_neg(tl + tr);
#pragma unroll
                for (int j = 0; j < CNT; ++j)
#pragma unroll
                    for (int r = 0; r < 16; ++r) acc[j][r] = acc[j][r] * fs.a * fs.b;
            }
            if (!last) {
                zero_padding();
                store_blocks(1.0f, 1.0f);
            }
            double ss = 0.0;
#pragma unroll
            for (int j = 0; j < CNT; ++j) ss += block_sumsq_all(acc[j]);
            ss = wave_sum_lane0(ss);
            if (lane == 0) red[wave] = ss;
            __builtin_amdgcn_s_waitcnt(0x0f70);  // the write-back is done
            __syncthreads();
            S = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) S += red[w];
            s = mul ? s + (double)eX + (double)eA : 2.0 * (s + (double)eX);
            eX = exponent_of_sumsq(S);
            if (last) break;
            tX = eX;
            if (eX < kPanelRawMinExp) {
                const PowScale f = pow2_neg(eX);
                store_blocks(f.a, f.b);
                __builtin_amdgcn_s_waitcnt(0x0f70);
                __syncthreads();
                tX = 0;
            }
        }
    }
    double sc = s;
    sc = sc > 4000.0 ? 4000.0 : (sc < -4000.0 ? -4000.0 : sc);
    const PowScale f = pow2_neg(eX);
#pragma unroll
    for (int j = 0; j < CNT; ++j)
        block_write_out(acc[j], bi[j], c0, n, out, scale != nullptr, f, (int)sc);
    if (scale && threadIdx.x == 0) *scale = (S == 0.0) ? 0.0 : s + (double)eX;
}

}  // namespace wgdetail

// A^p of one n x n matrix, 1 <= n <= NPMAX (64, 128 or 256), by the calling
// workgroup of NW = 8 or 16 waves, all of which must call it.  L0 and L1 hold
// WgPanelLds<NPMAX>::STAGE floats each (two distinct arrays), `red` NW
// doubles; `scratch` holds 2 * wg_npad(n)^2 floats of this workgroup's own
// memory, 16-byte aligned.  out may be A.  Contains barriers; returns with
// the workgroup synchronised.
template <int NPMAX, int NW>
__device__ __forceinline__ void wg_power_panel(const float *A, int n, int64_t p, float *out, double *scale,
                               float *scratch, float *L0, float *L1, double *red) {
    using namespace wgdetail;
    static_assert(NW == 8 || NW == 16, "block ranges are cut for 8 or 16 waves");
    static_assert(NPMAX == 64 || NPMAX == 128 || NPMAX == 256, "panel widths");
    constexpr int NT = NW * 64;
    constexpr int MB = (NPMAX / 32) * (NPMAX / 32) / NW > 0 ? (NPMAX / 32) * (NPMAX / 32) / NW : 1;
    static_assert(MB <= 4, "the dispatch below covers up to four blocks per wave");
    static_assert(NW == 16 || NPMAX <= 128, "the eight-wave piece table covers nb <= 4");
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double SA;
    int eA;
    if (!power_head<NT>(A, n, p, out, scale, red, &SA, &eA)) return;

    const int npad = wg_npad(n), nb = npad / 32;
    float *SX = scratch, *SAm = scratch + (size_t)npad * npad;
    const PowScale fa = pow2_neg(eA);
    copy_base_padded<NT>(A, n, npad, fa, [&](int r, int c, f4 v) {
        *(f4 *)(SAm + r * npad + c) = v;
    });
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();

    // this wave's piece of the block grid: cnt blocks from block row r0 of
    // block column c0
    const unsigned pc = NW == 16 ? kPieces16[nb - 1][wave] : kPieces8[nb - 1][wave];
    const int c0 = pc & 15, r0 = (pc >> 4) & 15, cnt = pc >> 8;
    // every wave takes part in the barriers of every product, whatever its count
#define MPOW_PANEL_CASE(C)                                                                          \
    case C:                                                                                         \
        if constexpr (C <= MB)                                                                      \
            panel_power_body<NPMAX, NW, C, (C < 1 ? 1 : C)>(A, n, p, out, scale, SX, SAm, L0, L1,   \
                                                            red, eA, c0, r0, wave);                 \
        break;
    switch (cnt) {
        MPOW_PANEL_CASE(0)
        MPOW_PANEL_CASE(1)
        MPOW_PANEL_CASE(2)
        MPOW_PANEL_CASE(3)
        MPOW_PANEL_CASE(4)
        default: break;
    }
#undef MPOW_PANEL_CASE
    __syncthreads();  // LDS, scratch and `red` may be reused by the caller
}

}  // namespace mpow
