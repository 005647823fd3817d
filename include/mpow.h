/*
 * mpow - integer matrix power A^p on AMD Instinct MI355X (gfx950).
 *
 * The operation is the one the paper computes in section 4: the p-th power of
 * a dense N x N matrix.  The paper's method (section 4.3) reaches A^p with a
 * number of matrix products logarithmic in p instead of the p-1 chained
 * products of the naive method (sections 4.1 and 4.2).  This library uses
 * left-to-right binary exponentiation: for every bit of p below the leading
 * one it squares the running matrix X <- X.X, and when that bit is set it
 * multiplies once more by the base, X <- X.A.  That is floor(log2 p) squarings
 * plus popcount(p)-1 multiplications, G(p) products in total.
 *
 * Range.  A^p leaves every floating-point range for the paper's powers (up to
 * 1024) unless A is scaled.  After each product the running matrix is scaled
 * by an exact power of two 2^-e, e = floor(log2 ||X||_F), and e is folded into
 * an integer log2 scale s carried in float64.  Scaling by a power of two is
 * exact, so it changes no rounding; it only keeps values in range.
 *
 * Conventions for every call below:
 *  - Matrices are float32, row-major, contiguous, n x n (element (i,j) at
 *    index i*n + j).  Matrix and scale pointers passed to run calls are
 *    DEVICE pointers on the plan's device, owned by the caller; the library
 *    never frees or keeps them past the call's completion on the stream.
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).  Run
 *    calls only enqueue work; they never synchronise with the host (the one
 *    exception: mpow_expm with squarings = -1 reads the input's norm back).
 *  - Every call returns an mpow_status; nothing throws across this boundary.
 *    Argument errors are detected on the host before anything is enqueued.
 *  - A plan is not thread-safe, and one plan must not have two runs in flight
 *    on different streams at once (they share its workspace).  Use one plan
 *    per concurrent stream.
 */
#ifndef MPOW_H
#define MPOW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mpow_status {
    MPOW_SUCCESS = 0,
    MPOW_ERR_INVALID = 1,     /* bad argument (null, n<1, n>max_n, p<0, overlap) */
    MPOW_ERR_UNSUPPORTED = 2, /* valid request the library does not implement */
    MPOW_ERR_NOMEM = 3,       /* device or pinned host allocation failed */
    MPOW_ERR_DEVICE = 4,      /* a HIP call failed; see mpow_last_device_error */
    MPOW_ERR_BUDGET = 5,      /* request can never fit the memory budget */
    MPOW_ERR_TIMEOUT = 6      /* a wait ended before the condition held */
} mpow_status;

/* Arithmetic of the matrix products.  Inputs and outputs are float32 in every
 * mode; scaling, the log2 scale and the final rescale are the same in all.
 *  MPOW_FP32   float32 MFMA products with float32 accumulation.
 *  MPOW_FP16X3 each scaled operand X' (X times an exact power of two that
 *              puts it in FP16 range) is split into FP16 hi = rn(X') and
 *              lo = rn(X' - hi); a product is hi.hi + hi.lo + lo.hi from
 *              three FP16 MFMA products accumulated in float32 (about
 *              float32 accuracy).
 *  MPOW_BF16X3 the same with BF16 halves (about 16 bits of operand
 *              precision; looser tolerance).
 *  MPOW_BF16X6 X' split into three BF16 parts x0 + x1 + x2 (about 24 bits);
 *              a product is the six BF16 MFMA products x_i y_j with
 *              i + j <= 2, accumulated in float32 (float32-level accuracy
 *              with float32's exponent range, after Henry, Tang and
 *              Heinecke, ARITH 2019). */
typedef enum mpow_mode {
    MPOW_FP32 = 0,
    MPOW_FP16X3 = 1,
    MPOW_BF16X3 = 2,
    MPOW_BF16X6 = 3
} mpow_mode;

/* Tolerance-driven mode choice (host only).  Every mode states an accuracy
 * bar: a result's relative Frobenius error against the exact power is at
 * most max(ABS, FACTOR * floor), where floor is the problem's own relative
 * sensitivity to float32-sized input noise (the change of A^p when every
 * entry of A moves by a relative +-2^-24; 0 for a well-conditioned power):
 *   MPOW_FP32, MPOW_FP16X3, MPOW_BF16X6   ABS 1e-5, FACTOR 64
 *   MPOW_BF16X3                           ABS 2e-4, FACTOR 1024
 * Returns the fastest mode whose bar is at most tol, in the order measured on
 * MI355X (n = 4096): BF16X3 (2.4x the FP32 rate), FP16X3 (2.3x), BF16X6
 * (1.35x), FP32.  wide_range != 0 skips FP16X3, whose parts lose entries
 * below about 2^-38 of the matrix's norm (FP16's range after scaling); the
 * BF16 modes keep float32's exponent range.  Returns -1 if no bar is met
 * (tol below 1e-5, or tol or floor negative or NaN). */
int mpow_mode_for_tolerance(double tol, double floor, int wide_range);

/* Plan flags. */
#define MPOW_FLAG_TIMING 1u /* record a pair of HIP events around every product
                               kernel launch; read with mpow_plan_timing.  The
                               two records add about 7 us per launch on
                               MI355X, as much as a whole product at n = 512:
                               leave it off where small-matrix latency counts */
#define MPOW_FLAG_POISON 2u /* testing: fill the workspace with NaN bytes at
                               creation instead of zeros, so a read of memory
                               the run has not written shows in the result */
#define MPOW_FLAG_EXPM 4u   /* also allocate what mpow_expm needs: one more
                               max_n x max_n float32 buffer (FP32 plans) */
#define MPOW_FLAG_WINDOW 8u /* FP32 plans: mpow_run follows the sliding-window
                               schedule (mpow_window_schedule, w = 2 or 3) when
                               it takes fewer products than binary; holds four
                               more max_n x max_n buffers (A^2, A^3, A^5, A^7).
                               Results then differ from the binary schedule's
                               in rounding (same tolerance). */
#define MPOW_FLAG_SPLIT_PASS 16u /* BF16 modes: split each product's result into
                               its BF16 parts in a separate pass (a float32
                               write, a read and a launch per product) instead
                               of in the product's epilogue; the same results
                               bit for bit, for comparison and measurement */

/* Upper bound on the number of products of one power (p < 2^63 needs <= 124). */
#define MPOW_MAX_STEPS 126

/* Largest p mpow_run_naive accepts. */
#define MPOW_NAIVE_MAX_P 4096

typedef struct mpow_plan *mpow_plan_t;

/* Static description of a status code.  Never NULL. */
const char *mpow_status_str(int status);

/* G(p) = floor(log2 p) + popcount(p) - 1 for p >= 2, 0 for p in {0,1},
 * -1 for p < 0.  Host only; never touches a device. */
int mpow_gemm_count(int64_t p);

/* Writes the product schedule of p (section 4.3, left-to-right binary
 * exponentiation) into ops[0..G(p)-1]: 0 = square X <- X.X, 1 = multiply
 * X <- X.A.  Returns G(p), or -1 if p < 0, ops is NULL while G(p) > 0, or
 * cap < G(p).  Host only. */
int mpow_schedule(int64_t p, uint8_t *ops, int cap);

/* Sliding-window schedule of p >= 1 (host only; an extension beyond the paper:
 * fewer products than binary exponentiation when p has long runs of ones,
 * e.g. 27 instead of 38 for p = 2^20 - 1).  Windows of up to w bits, w in
 * 1..3 (1 is the binary schedule of section 4.3), or w = 0 for the w with
 * the fewest products.  The bits of p are read from the top; a zero bit
 * squares the running matrix, a window (a run of at most w bits starting and
 * ending with a one, value v) squares it once per bit and multiplies it by
 * the precomputed odd power A^v; the first window starts from A^v.  Matrix
 * slots: 0 = A, 1 = A^2, 2 = A^3, 3 = A^5, 4 = A^7, 5 and 6 = the running
 * matrix.  Product k computes slot ops[3k] = slot ops[3k+1] . slot
 * ops[3k+2]; *result receives the slot that holds A^p.  Returns the number
 * of products (ops may be NULL to count only), or -1 (p < 1, w outside
 * 0..3, result NULL, or cap too small). */
int mpow_window_schedule(int64_t p, int w, uint8_t *ops, int cap, int *result);

/* Device bytes a plan for (max_n, max_batch, mode) allocates without the
 * optional buffers of MPOW_FLAG_EXPM (max_n^2 floats) and MPOW_FLAG_WINDOW
 * (four max_n^2 float matrices and their per-tile partial sums); 0 for
 * invalid arguments.  The batch part is sized for 256 CUs.  Host only. */
size_t mpow_workspace_bytes(int max_n, int max_batch, int mode);

/* Creates a plan on HIP device `device` for matrices up to max_n x max_n and
 * batches of up to max_batch matrices (0: no batched calls).  All device
 * workspace is allocated here, never on the run path.  `mode` is an
 * mpow_mode.  On success *plan owns the workspace until mpow_plan_destroy.
 * Errors: INVALID (plan NULL, max_n < 1, max_batch < 0, unknown mode/flags),
 * UNSUPPORTED (MPOW_FLAG_WINDOW with a mode other than MPOW_FP32), DEVICE (no
 * such device / HIP failure),
 * NOMEM (allocation failed; nothing is leaked). */
mpow_status mpow_plan_create(mpow_plan_t *plan, int device, int max_n, int max_batch,
                             int mode, uint32_t flags);

/* Frees the plan's workspace after waiting for the device to finish work
 * that uses it.  NULL is accepted and ignored. */
mpow_status mpow_plan_destroy(mpow_plan_t plan);

/* A^p (sections 4.3 and 4.1 for the definition).
 *   A          device, n*n float32, read only.
 *   n          1 <= n <= the plan's max_n.
 *   p          p >= 0.  p = 0 gives the identity (also for singular A),
 *              p = 1 gives A.
 *   out        device, n*n float32, written.  It may be the same pointer as
 *              A; any other overlap with A is INVALID.
 *   log2_scale NULL: out = A^p rounded to float32 (entries beyond float32
 *              range become +-inf or 0).  Non-NULL (device, one double):
 *              out = M and *log2_scale = s with A^p = M * 2^s and
 *              ||M||_F in [1, 2); s is an integer held in a double.  A zero
 *              result (zero A, or a power of a nilpotent A that vanishes)
 *              gives M = 0 and s = 0.
 * NaN or Inf entries propagate into the result (status is still SUCCESS).
 * Errors: INVALID (arguments), DEVICE (launch failure). */
mpow_status mpow_run(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                     double *log2_scale, void *stream);

/* The paper's naive method (sections 4.1 and 4.2): A^p by p - 1 chained
 * products X <- X.A (the same float32 product kernels, scaling and output
 * convention as mpow_run), for comparing against the logarithmic schedule.
 * Arguments as mpow_run; p must be <= MPOW_NAIVE_MAX_P.  Errors: INVALID
 * (also p > MPOW_NAIVE_MAX_P), UNSUPPORTED (plan mode other than MPOW_FP32),
 * DEVICE. */
mpow_status mpow_run_naive(mpow_plan_t plan, const float *A, int n, int64_t p, float *out,
                           double *log2_scale, void *stream);

/* Largest n mpow_run_noalloc accepts. */
#define MPOW_NOALLOC_MAX_N 2048

/* mpow_run without a plan and without any device allocation, for callers
 * that cannot allocate device memory: code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc.  It computes what
 * mpow_run does on a float32 plan with default kernels (the same kernels,
 * so the same bits), on the CURRENT device; `stream` must belong to it
 * (NULL: the null stream).
 * Workspace: a fixed device array of about 32 MiB (the float32 workspace
 * of a 2048 x 2048 power) inside the library, one per GPU, held from the
 * library's first use on that GPU until the process ends.  The first call
 * on a device looks up that device's copy (no allocation); no call
 * allocates or frees device or pinned memory.
 * Concurrency: every call on one GPU shares that GPU's array, so two calls
 * whose work overlaps on the device (different streams, not ordered by
 * events) race and give undefined results; calls on one stream, or ordered
 * by events, are safe.  Nothing in the array needs clearing between calls.
 * Arguments as mpow_run (A, out, log2_scale device pointers, out may be A).
 * Errors: INVALID (arguments, or a stream of another device), UNSUPPORTED
 * (n > MPOW_NOALLOC_MAX_N; nothing enqueued), DEVICE (HIP failure). */
mpow_status mpow_run_noalloc(const float *A, int n, int64_t p, float *out, double *log2_scale,
                             void *stream);

/* Matrix exponential e^A by scaling and squaring, float32 products (the
 * power's kernels; an extension beyond the paper, whose subject is A^p):
 * e^A = (e^B)^(2^j) with B = A * 2^-j exact; e^B is the degree-8 Taylor
 * polynomial by Horner's rule, I + B(I + B/2(... (I + B/8))), with
 * ||B||_F < 1/2 (remainder below float32 resolution) when j is chosen from
 * the norm; the j squarings are the power T^(2^j) of mpow_run.
 *   A, n, out, log2_scale   as for mpow_run (out = M and *log2_scale = s
 *              with e^A = M * 2^s, or out = e^A rounded to float32).
 *   squarings  j in 0..62, or -1: j = max(0, floor(log2 ||A||_F) + 2),
 *              0 for a zero or non-finite norm.  Choosing j reads the norm
 *              back to the host: the call then waits for `stream` once.
 * The plan must be a MPOW_FP32 plan created with MPOW_FLAG_EXPM.  Errors:
 * INVALID (arguments, squarings outside -1..62), UNSUPPORTED (other plan,
 * or -1 with ||A||_F >= 2^61), DEVICE. */
mpow_status mpow_expm(mpow_plan_t plan, const float *A, int n, float *out, double *log2_scale,
                      int squarings, void *stream);

/* `count` independent powers in one call: matrix i is A[i] (device pointer,
 * n[i] x n[i]) raised to p[i] into out[i], with log2_scale[i] as in mpow_run
 * (log2_scale itself may be NULL: no scales for any matrix).  A, n, p and out
 * are HOST arrays of length count.  Per-matrix semantics equal mpow_run's.
 * Errors: INVALID (count < 0 or > max_batch, any per-matrix argument invalid,
 * n[i] > 256), DEVICE. */
mpow_status mpow_run_batched(mpow_plan_t plan, int count, const float *const *A, const int *n,
                             const int64_t *p, float *const *out, double *log2_scale,
                             void *stream);

/* Tile table of the batched kernel: table[b] is the tile shape used for
 * matrices with n in (16(b-1), 16b], b = 1..16 (table[0] is unused).
 * Shapes 0 = 128x128, 1 = 64x64, 2 = 256x256 on 8 waves: each product is
 * tiled, the running matrices pass through per-worker scratch in memory.
 * Shapes 3 and 4: one workgroup computes the matrix's whole power with
 * every product held in its accumulators (section 4.3's schedule with the
 * operands staged in local memory, section 4.3.2); 3 keeps the base and the
 * running matrix resident in LDS for n <= 128 (four waves and 32 KB up to
 * n = 64, eight waves and 128 KB above) and streams K panels of both from
 * scratch for n > 128; 4 always streams K panels (64 KB of LDS, two
 * workgroups per CU, up to n = 128; 128 KB above).  Every shape gives
 * bit-identical results wherever no intermediate value is subnormal (the
 * shapes apply the same power-of-two scales at different points of a
 * product); only speed differs.  A batch runs as one launch
 * per group of matrices that share a kernel instance (at most five, in
 * order on the stream): the tiled shapes on the smallest instance that
 * holds every tiled shape used (without shape 0 or 2: a 64x64-only instance
 * that keeps four workgroups per CU; with shape 2: one 8-wave workgroup per
 * CU; with shape 0 and every such matrix allowing 16-byte loads, n % 4 == 0
 * and a 16-byte aligned A, the instance whose tiles load straight into
 * LDS), and each whole-power form on its own instance.
 * A plan starts with shape 4 for every size (on MI355X the fastest at every
 * size of uniform batches and on ragged batches); mpow_plan_autotune may
 * replace it with measured choices.
 * set = 0 copies the plan's table into table[0..16]; set = 1 replaces it.
 * len must be >= 17.
 * Errors: INVALID (plan NULL or without batch support, len < 17, a shape
 * outside 0..4). */
mpow_status mpow_plan_tile_table(mpow_plan_t plan, int *table, int len, int set);

#define MPOW_TUNE_FORCE 1u /* ignore an existing cache file */

/* Autotuner (precedent: the per-problem tile choice of section 4.3.7).
 * Every plan: for each 256-wide size bucket n = 256 b up to
 * min(max_n, 8192) (from n = 768 for MPOW_FP32, whose smaller sizes keep the
 * whole-K tile), times one product (a power A^2) on each product kernel of
 * the plan's mode that adds the products in the per-size default's order
 * (float32: the LDS-DMA 256x128, 256x256, 128x128 and 64x64 tiles; split
 * modes: the 128x128 and 256x256 tiles) and keeps the fastest for sizes of
 * that bucket, for 16-byte-loadable inputs (float32) or all inputs (split
 * modes); results are bit for bit those of the default picks.
 * MPOW_FP32 plans with batch support also tune the batched kernel's tile
 * table: every size bucket up to min(max_n, 256) times each of the five tile
 * shapes on a synthetic batch of that size that fills all workers twice
 * (p = 100, eight products), run through mpow_run_batched's own grouping and
 * launches; because a mixed batch runs one launch per kernel instance it
 * needs, one after another, whole tables are then timed on a synthetic
 * ragged batch (sizes uniform over the buckets, p log-uniform in [2, 1000]):
 * the per-bucket winners, the table before tuning, and each single shape for
 * all sizes; the fastest becomes the plan's tile table.
 * Timing starts after a few tenths of a second of warm-up work (an idle GPU
 * runs at a lower clock at first), and the candidates of each choice are
 * timed round-robin, each keeping its fastest run.
 * If cache_path is non-NULL and holds choices written for the same GPU model
 * (architecture and CU count) and mode that cover everything this plan tunes,
 * they are loaded instead (unless MPOW_TUNE_FORCE); otherwise the fresh
 * choices are written there.  Synchronous; allocates temporary device memory
 * (not on the run path).  Errors: INVALID (plan NULL, unknown flags), NOMEM,
 * DEVICE. */
mpow_status mpow_plan_autotune(mpow_plan_t plan, const char *cache_path, uint32_t flags);

/* The product kernel (an MPOW_KERNEL_* id) mpow_run on this plan uses at size
 * n: the forced kernel, else the autotuned pick for n's size bucket, else the
 * per-size default; MPOW_KERNEL_POWER_WG where the whole power runs in one
 * workgroup (float32 plans without MPOW_FLAG_WINDOW; window plans report the
 * product kernel of their window schedules).  aligned != 0: a 16-byte
 * aligned input.  Host only.  -1 for a NULL plan or n outside 1..max_n. */
int mpow_plan_kernel_for(mpow_plan_t plan, int n, int aligned);

/* Forces the product kernel that mpow_run / mpow_run_naive use on this plan
 * for every n (kernel: an MPOW_KERNEL_* id of the plan's mode), or restores
 * the per-size default (kernel = -1).  The float32 kernels that load their
 * tiles straight into LDS (the 256x256 kernel and the ..._DMA kernels) need
 * n % 4 == 0 and a 16-byte aligned A; otherwise (and for the ..._DMA
 * kernels also when n > 23170) the 128x128 kernel runs instead (the 64x64
 * kernel for MPOW_KERNEL_GEMM_F32_64_DMA).  Kernels without a K split give
 * bit-identical results; a K-split kernel (..._K2/_K4/_K8) adds its partial
 * sums in its own fixed order, so its results are deterministic but may
 * differ from the others in the last bits.  Not for use while a run on the plan is enqueued
 * from another thread.  Errors: INVALID (plan NULL, kernel not of the plan's
 * mode). */
mpow_status mpow_plan_set_kernel(mpow_plan_t plan, int kernel);

/* The float32 product kernel (an MPOW_KERNEL_* id) that mpow_run uses at
 * size n when no kernel is forced: aligned != 0 means a 16-byte aligned A
 * (the LDS-DMA tiles need that and n % 4 == 0).  Host-only, no device call;
 * -1 for n < 1.  Below n = 768 the 32x32 tile with a K split: for a
 * 16-byte-loadable input up to n = 512 its whole-K-in-LDS form over 8 waves,
 * otherwise the register-staged form over 4 waves; from n = 768 the LDS-DMA tile with the
 * best estimated rate for how its tile count fills the 256 CUs in whole
 * waves (section 4.3.7's tiled product, tile size chosen per n).  For
 * n <= 64 mpow_run's binary schedule does not launch a product kernel at
 * all: it runs the whole power in one workgroup (MPOW_KERNEL_POWER_WG); the
 * kernel returned here is then the one of its naive and window forms. */
int mpow_fp32_kernel_for(int n, int aligned);

/* The last hipError_t value a call on this plan saw (0 if none): the HIP
 * error behind an MPOW_ERR_DEVICE status (the "last HIP error" query of this
 * boundary; a server reports its own in mpow_srv_stats).  Host only. */
int mpow_last_device_error(mpow_plan_t plan);

/* Kernel identifiers for timing queries. */
enum {
    MPOW_KERNEL_GEMM_F32_128 = 0, /* float32 product, 128x128 tiles */
    MPOW_KERNEL_GEMM_F32_64 = 1,  /* float32 product, 64x64 tiles */
    MPOW_KERNEL_GEMM_F32_32 = 2,  /* float32 product, 32x32 tiles */
    MPOW_KERNEL_GEMM_F16X3_128 = 3,  /* FP16 hi/lo three-product, 128x128 tiles */
    MPOW_KERNEL_GEMM_BF16X3_128 = 4, /* BF16 hi/lo three-product, 128x128 tiles */
    MPOW_KERNEL_GEMM_F32_256 = 5,    /* float32 product, 256x256 tiles, 8 waves, LDS-DMA loads */
    MPOW_KERNEL_GEMM_F32_128x64 = 6, /* float32 product, 128x64 tiles */
    MPOW_KERNEL_GEMM_F16X3_256 = 7,  /* FP16 hi/lo three-product, 256x256 tiles, 8 waves */
    MPOW_KERNEL_GEMM_BF16X3_256 = 8, /* BF16 hi/lo three-product, 256x256 tiles, 8 waves */
    MPOW_KERNEL_GEMM_F32_32_K4 = 9,  /* float32 product, 32x32 tiles, K split over 4 waves */
    MPOW_KERNEL_GEMM_F32_32_K8 = 10, /* float32 product, 32x32 tiles, K split over 8 waves */
    MPOW_KERNEL_GEMM_F32_64_K2 = 11, /* float32 product, 64x64 tiles, 2x2 waves, K split in 2 */
    MPOW_KERNEL_GEMM_F32_128_K2 = 12, /* float32 product, 128x128 tiles, 2x2 waves, K split in 2 */
    MPOW_KERNEL_GEMM_BF16X6_128 = 13, /* BF16 three-part six-product, 128x128 tiles */
    MPOW_KERNEL_GEMM_BF16X6_256 = 14, /* BF16 three-part six-product, 256x256 tiles, 8 waves */
    MPOW_KERNEL_GEMM_F32_64_DMA = 15,  /* float32 product, 64x64 tiles, LDS-DMA loads, K tile 32 */
    MPOW_KERNEL_GEMM_F32_128_DMA = 16, /* float32 product, 128x128 tiles, 4x2 waves, LDS-DMA, K tile 32 */
    MPOW_KERNEL_GEMM_F32_256x128_DMA = 17, /* float32 product, 256x128 tiles, 4x2 waves, LDS-DMA */
    MPOW_KERNEL_GEMM_F32_32_K4_DMA = 18, /* float32 product, 32x32 tiles, K split over 4 waves, whole K in LDS (n <= 512) */
    MPOW_KERNEL_POWER_WG = 19, /* float32, n <= 128: the whole power in one launch of one
                                  8-wave workgroup, base and running matrix resident in
                                  LDS (mpow_run only, its default for n <= 64; timing
                                  counts G(p) 2 n^3 per launch) */
    MPOW_KERNEL_GEMM_F32_32_K8_DMA = 20, /* float32 product, 32x32 tiles, K split over 8 waves, whole K in LDS (n <= 512) */
    MPOW_KERNEL_COUNT = 21
};

/* Timing of product launches recorded under MPOW_FLAG_TIMING since the last
 * reset: number of launches, summed event-measured milliseconds and summed
 * algorithmic flops (2 n^3 per product).  Waits for the recorded events.
 * The name written to *name (may be NULL) is the kernel's symbol name.
 * Errors: INVALID (plan NULL, flag not set, bad kernel id), DEVICE. */
mpow_status mpow_plan_timing(mpow_plan_t plan, int kernel, int64_t *launches, double *total_ms,
                             double *total_flop, const char **name);
mpow_status mpow_plan_timing_reset(mpow_plan_t plan);

/* ------------------------------------------------------------------------
 * Request server (continuous batching).
 *
 * An engine thread owns a device-memory arena of hbm_budget bytes, n_streams
 * HIP streams and a ragged-batch context.  Requests are independent powers
 * (the same operation as mpow_run) of mixed n, p and mode:
 *  - float32 requests with n <= 256 (and max_batch > 0) wait in one FIFO and
 *    leave together, up to max_batch at a time, as one persistent batched
 *    launch whenever fewer than two batches are in flight (one running, one
 *    queued behind it); requests arriving meanwhile join the next batch.
 *  - every other request is admitted in arrival order once its workspace
 *    (mpow_workspace_bytes(n, 0, mode)) fits the unused part of the arena and
 *    one of the streams has fewer than 2 requests in flight; it then runs on
 *    that stream, its operands and partial powers staying in its arena
 *    region, overlapping with the other streams and the batch.
 * Results do not depend on what else runs: every request's kernels and their
 * accumulation order depend only on (n, mode).
 * ------------------------------------------------------------------------ */
typedef struct mpow_srv *mpow_srv_t;

typedef struct mpow_completion {
    uint64_t id;
    int32_t status;  /* MPOW_SUCCESS or MPOW_ERR_DEVICE */
    int32_t route;   /* 0: own stream, 1: batched */
    double t_submit; /* seconds since server creation (host steady clock) */
    double t_start;  /* when the engine enqueued its work */
    double t_end;    /* when the engine saw its completion event */
} mpow_completion;

typedef struct mpow_srv_stats_t {
    uint64_t submitted, completed, rejected;
    int32_t queued, in_flight;
    size_t arena_capacity, arena_in_use, arena_peak;
    int32_t last_device_error;
    int32_t pad;
} mpow_srv_stats_t;

/* Creates a server on `device` for matrices up to max_n, with an arena of
 * hbm_budget bytes (allocated here), n_streams streams (1..64) and batches of
 * up to max_batch small requests (0: no batching).  flags must be 0.
 * Errors: INVALID, DEVICE, NOMEM. */
mpow_status mpow_srv_create(mpow_srv_t *srv, int device, int max_n, size_t hbm_budget,
                            int n_streams, int max_batch, uint32_t flags);

/* Queues A^p (device pointers as in mpow_run; A and out must stay valid and
 * untouched until the request completes).  Never blocks on the device.
 * *id (may be NULL) receives the request id.  Errors: INVALID (arguments,
 * n > max_n, server stopping), BUDGET (its workspace exceeds the whole
 * arena: it could never run). */
mpow_status mpow_srv_submit(mpow_srv_t srv, const float *A, int n, int64_t p, int mode, float *out,
                            double *log2_scale, uint64_t *id);

/* Moves up to max completion records into out (oldest first); returns their
 * number, or -1 for bad arguments. */
int mpow_srv_poll(mpow_srv_t srv, mpow_completion *out, int max);

/* Blocks until every submitted request has completed, or timeout_s passes
 * (TIMEOUT). */
mpow_status mpow_srv_wait_idle(mpow_srv_t srv, double timeout_s);

mpow_status mpow_srv_stats(mpow_srv_t srv, mpow_srv_stats_t *stats);

/* Stops accepting requests, lets the engine finish every queued and running
 * one, then frees everything.  NULL is accepted. */
mpow_status mpow_srv_destroy(mpow_srv_t srv);

/* CPU-only run of the same admission and batching policy against a simulated
 * executor (no device is touched): each stream runs its requests one after
 * another at plain_flops; batches (at most two in flight) run one after
 * another, each taking launch_overhead_s plus its flops at batch_flops; a
 * request costs launch_overhead_s plus 2 G(p) n^3 flops.
 * reqs must be sorted by t_arrive.  results[i] receives the status (SUCCESS or
 * BUDGET), route, stream and simulated admission/start/end times of request i;
 * *peak_bytes the largest arena use.  Errors: INVALID; BUDGET if the policy
 * ever exceeded the budget (a bug). */
typedef struct mpow_sim_config {
    size_t hbm_budget;
    int32_t n_streams, depth, batch_cap, pad;
    double plain_flops, batch_flops, launch_overhead_s;
} mpow_sim_config;
typedef struct mpow_sim_request {
    double t_arrive;
    int32_t n, mode;
    int64_t p;
} mpow_sim_request;
typedef struct mpow_sim_result {
    int32_t status, route, stream, pad;
    double t_admit, t_start, t_end;
} mpow_sim_result;
mpow_status mpow_srv_simulate(const mpow_sim_config *cfg, const mpow_sim_request *reqs, int count,
                              mpow_sim_result *results, size_t *peak_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MPOW_H */
