// Device bodies of the memory-bound steps of a power (the input's sum of
// squares and the final rescale), used by their stand-alone kernels.
#pragma once

#include "scale_device.h"

namespace mpow {

// Sum of squares (float64) of A[begin, end) by one workgroup of NT threads:
// per-thread sums in a fixed element order, then a fixed tree over `red`
// (NT doubles of LDS).  VEC: 16-byte loads (begin a multiple of 4, A 16-byte
// aligned), four in flight per thread.  Returns the sum to every thread.
template <int NT, bool VEC>
__device__ __forceinline__ double sumsq_range(const float *__restrict__ A, int64_t begin,
                                              int64_t end, double *red) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    double acc = 0.0;
    if (VEC && begin < end) {
        const f4v *V = (const f4v *)A;
        const int64_t b4 = begin / 4, e4 = end / 4;
        int64_t i = b4 + threadIdx.x;
        for (; i + 3 * NT < e4; i += 4 * NT) {
            f4v v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = V[i + u * NT];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc += (double)v[u][c] * (double)v[u][c];
        }
        for (; i < e4; i += NT) {
            const f4v v = V[i];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc += (double)v[c] * (double)v[c];
        }
        // the last 1-3 elements when the range does not end on a multiple of 4
        for (int64_t j = e4 * 4 + threadIdx.x; j < end; j += NT) {
            const double v = (double)A[j];
            acc += v * v;
        }
    } else if (!VEC) {
        for (int64_t i = begin + threadIdx.x; i < end; i += NT) {
            const double v = (double)A[i];
            acc += v * v;
        }
    }
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

// Final rescale of elements first, first + stride, ... of the n x n matrix:
// with_scale: out = C * 2^-eG (exact power-of-two scaling);
// otherwise : out = ldexp(C, sG) in float64, rounded to float32 (sG clamped
//             to +-4000, beyond which every float32 result is 0 or inf).
// The 16-byte path (n^2 % 4 == 0, C and out 16-byte aligned) counts first and
// stride in groups of four elements.  C and out may be the same buffer.
__device__ __forceinline__ void finish_range(const float *C, float *out, int n, bool with_scale,
                                             int eG, double sG, int64_t first, int64_t stride) {
    typedef float f4v __attribute__((ext_vector_type(4)));
    const int64_t total = (int64_t)n * n;
    const bool vec = (total % 4 == 0) && ((((uintptr_t)C) | ((uintptr_t)out)) & 15) == 0;
    if (with_scale) {
        const PowScale f = pow2_neg(eG);
        if (vec) {
            for (int64_t i = first; i < total / 4; i += stride)
                ((f4v *)out)[i] = ((const f4v *)C)[i] * f.a * f.b;
        } else {
            for (int64_t i = first; i < total; i += stride) out[i] = C[i] * f.a * f.b;
        }
    } else {
        sG = sG > 4000.0 ? 4000.0 : (sG < -4000.0 ? -4000.0 : sG);
        const int si = (int)sG;
        if (vec) {
            for (int64_t i = first; i < total / 4; i += stride) {
                const f4v c = ((const f4v *)C)[i];
                f4v o;
#pragma unroll
                for (int k = 0; k < 4; ++k) o[k] = (float)ldexp((double)c[k], si);
                ((f4v *)out)[i] = o;
            }
        } else {
            for (int64_t i = first; i < total; i += stride) out[i] = (float)ldexp((double)C[i], si);
        }
    }
}

}  // namespace mpow
