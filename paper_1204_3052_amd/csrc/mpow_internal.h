// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/mpow.h"

namespace mpow {

// ---------------------------------------------------------------- workspace

// Device memory one power needs (plan-owned, or carved from a server arena).
//  buf[0], buf[1]   ping-pong running matrices, n^2 floats each
//  part[0], part[1] per-tile partial sums of squares of buf[0] / buf[1]
//  partA            per-block partial sums of squares of the input A
//  escale           escale[k] = floor(log2 ||C_k||_F) of the k-th product's
//                   output (C_0 = A), written by the kernel that consumes C_k
//  sx, sa           split modes: 16-bit hi/lo of the running matrix and of A
//                   (row-major hi, lo, then transposed hi, lo), ld x ld each
// Size buckets of the tuned product-kernel picks: n in (256 (b - 1), 256 b]
// for b = 1 .. kPickBuckets - 1 (up to n = 8192).
constexpr int kPickBuckets = 33;

struct Workspace {
    float *buf[2] = {nullptr, nullptr};
    double *part[2] = {nullptr, nullptr};
    double *partA = nullptr;
    int *escale = nullptr;
    // split parts of the running matrix (sx) and of A (sa): [0] row-major,
    // [1] transposed, part k = 0 .. split_parts(mode) - 1
    void *sx[2][3] = {};
    void *sa[2][3] = {};
    // BF16 modes (fused split): a second set of the running matrix's parts,
    // so that a product writes the next operand's parts while it reads its own
    void *sy[2][3] = {};
    bool split_pass = false;  // BF16 modes: the separate split pass (MPOW_FLAG_SPLIT_PASS)
    int max_n = 0;
    int mode = MPOW_FP32;
    int kernel = -1;  // product kernel forced for every size, -1: per-size default
    // product kernel measured fastest by mpow_plan_autotune for n in
    // (256 (b - 1), 256 b], stored as id + 1 (0: none, the per-size default)
    int8_t pick1[kPickBuckets] = {};
    // window schedules (plans with MPOW_FLAG_WINDOW): A^2, A^3, A^5, A^7 with
    // their partial sums, and the right operand's exponent of every product
    float *wp[4] = {};
    double *wpart[4] = {};
    int *escaleY = nullptr;
};

size_t round_up(size_t x, size_t a);

// Pieces of the workspace layout (each 256-byte aligned): a running matrix,
// its per-tile partial sums (the smallest product tile is 32 x 32), the
// input's partial sums, and the per-product exponents.
constexpr size_t ws_align(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t ws_buf_bytes(int max_n) { return ws_align((size_t)max_n * (size_t)max_n * 4); }
constexpr size_t ws_part_bytes(int max_n) {
    return ws_align(((size_t)max_n + 31) / 32 * (((size_t)max_n + 31) / 32) * 8);
}
constexpr int kMaxNormBlocks = 1024;  // partial sums of A (capacity of Workspace::partA)
constexpr size_t ws_partA_bytes() { return ws_align((size_t)kMaxNormBlocks * 8); }
constexpr size_t ws_escale_bytes() { return ws_align(((size_t)MPOW_NAIVE_MAX_P + 2) * 4); }
// Bytes of a float32 workspace for matrices up to max_n.
constexpr size_t fp32_workspace_bytes(int max_n) {
    return 2 * ws_buf_bytes(max_n) + 2 * ws_part_bytes(max_n) + ws_partA_bytes() + ws_escale_bytes();
}

// Bytes of one workspace for matrices up to max_n in `mode` (256-aligned).
size_t workspace_bytes(int max_n, int mode);
// Lays a workspace out over [base, base + workspace_bytes(max_n, mode)).
void workspace_carve(char *base, int max_n, int mode, Workspace *ws);

// ---------------------------------------------------------------- timing

struct TimingRecord {
    int kernel;
    double flop;
    hipEvent_t start, stop;
};

// Optional HIP-event timing of product launches (MPOW_FLAG_TIMING).
struct TimingSink {
    std::vector<hipEvent_t> free_events;
    std::vector<TimingRecord> pending;
    int64_t launches[MPOW_KERNEL_COUNT] = {};
    double ms[MPOW_KERNEL_COUNT] = {};
    double flop[MPOW_KERNEL_COUNT] = {};
    hipError_t start(int kernel, double flop, hipStream_t s, TimingRecord *rec);
    hipError_t stop(TimingRecord *rec, hipStream_t s);
    hipError_t collect();  // waits for pending records and accumulates them
    void reset();
    void destroy();
};

// Sliding-window product schedules (float32 plans with MPOW_FLAG_WINDOW).
// Matrix slots: A, A^2, A^3, A^5, A^7, and the running matrix's two buffers.
constexpr int kSlotA = 0, kSlotA2 = 1, kSlotR0 = 5, kSlotR1 = 6, kSlots = 7;
// Products of the window schedule of p with windows of up to w bits (1..3):
// ops[3k], ops[3k+1], ops[3k+2] = destination, left and right slot of
// product k (ops may be NULL to count); *result = the slot holding A^p.
// Returns the number of products, -1 on bad arguments or cap too small.
int window_schedule(int64_t p, int w, uint8_t *ops, int cap, int *result);

// A window schedule as a kernel argument.
constexpr int kMaxGraphOps = 128;
struct GraphOps {
    uint8_t op[kMaxGraphOps][3];  // dst, x, y slots of product k
    int count;
    int result;                   // the slot holding A^p
};
hipError_t launch_finish_graph(const float *C, int n, const double *partC, int nPartC,
                               const int *eX, const int *eY, const GraphOps &g, float *out,
                               double *log2_scale, hipStream_t s);

// Enqueues A^p on stream s using workspace ws (ws.max_n >= n, ws.mode = mode).
// Arguments must already be validated.  Returns the first HIP error.
hipError_t enqueue_power(const Workspace &ws, const float *A, int n, int64_t p, float *out,
                         double *log2_scale, hipStream_t s, TimingSink *timing);
// Matrix exponential: e^A = (Taylor-8 of 2^-j A)^(2^j) with T (n*n floats,
// not part of ws) holding the Taylor polynomial; 0 <= j <= 62.
hipError_t enqueue_expm(const Workspace &ws, float *T, const float *A, int n, int j, float *out,
                        double *log2_scale, hipStream_t s, TimingSink *timing);
// floor(log2 ||A||_F) into *dev_e (INT_MIN for a zero or non-finite norm).
hipError_t enqueue_norm_exponent(const Workspace &ws, const float *A, int n, int *dev_e,
                                 hipStream_t s);
int expm_squarings_for(int e);  // max(0, e + 2); 0 for INT_MIN
// The whole power of one n x n matrix (n <= kPowerWgMaxN) in a single launch
// of one workgroup that keeps its operands in LDS (power_wg.h).
constexpr int kPowerWgMaxN = 128;
hipError_t launch_power_wg(const float *A, int n, int64_t p, float *out, double *log2_scale,
                           hipStream_t s);
// mpow_run's float32 path takes launch_power_wg for n up to this size unless
// a product kernel is forced.  Measured per power (p = 64 / 1000): n = 16-64
// one workgroup takes 19-46 us against 40-88 us for one launch per product;
// at n = 96 and 128 it is slower (53 / 83 us against 43 / 42 us at p = 64),
// because one CU's MFMA rate bounds it (a 128^3 product is 6.8 us on one CU
// at peak, about what a launched product costs on many CUs).
constexpr int kPowerWgAutoMaxN = 64;
// The naive method: p - 1 chained float32 products X <- X.A (p <= MPOW_NAIVE_MAX_P).
hipError_t enqueue_power_naive(const Workspace &ws, const float *A, int n, int64_t p, float *out,
                               double *log2_scale, hipStream_t s, TimingSink *timing);

// ---------------------------------------------------------------- kernels

// How one float32 product kernel is launched.
struct GemmLaunch {
    const float *X;          // left operand (scaled by 2^-eX on load)
    const double *partX;     // partial sums of squares of X
    int nPartX;
    const float *Y;          // right operand (scaled by 2^-eY on load)
    const double *partY;
    int nPartY;
    float *C;                // output, n x n
    double *partC;           // output partials, one per tile
    int *eSlot;              // where block 0 records eX (may be null)
    int n;
    int *eSlotY = nullptr;   // where block 0 records eY (may be null)
    // partX / partY null: the operand's exponent is eXfix / eYfix instead
    int eXfix = 0, eYfix = 0;
    // non-null: eY is read from here (recorded by an earlier launch on the
    // stream) instead of being reduced from partY
    const int *eYin = nullptr;
    float alpha = 1.0f;      // the identity-adding epilogue: C = alpha X'Y' + I
    // non-null (X = Y = normA, n % 4 == 0, 16-byte aligned; the whole-K
    // 32 x 32 kernels only): each workgroup sums normA's squares itself, in
    // one fixed order, for eX = eY, instead of reducing partials of a
    // separate launch
    const float *normA = nullptr;
};

// Largest n for which the first product of a float32 power reduces the
// input's norm itself (GemmLaunch::normA): every workgroup reads the whole
// input once more, n^2 floats.
constexpr int kNormInKernelMaxN = 256;

// Split of a float32 matrix into 16-bit hi/lo, row-major and transposed,
// zero-padded to ld x ld.
struct SplitLaunch {
    const float *X;
    const double *part;   // partial sums of squares of X
    int nPart;
    int n, ld;
    void *rm[3], *tr[3];  // parts, row-major and transposed (ld x ld each)
    int *eSlot;           // block (0,0) records e of X here (may be null)
};

// Split-precision product: C = (X'Y') * 2^-2k from the operands' parts.
struct SplitGemmLaunch {
    const void *x[3];  // left operand's parts, row-major, ld
    const void *y[3];  // right operand's parts, transposed, ld
    float *C;          // float32 output (unused when the parts are written)
    double *partC;
    int n, ld;
    // Fused split (BF16 modes): operands whose parts are those of an
    // unnormalised matrix carry its partial sums of squares; the product is
    // scaled by 2^-(eX + eY) in the epilogue (null: exponent 0).
    const double *partX = nullptr;
    int nPartX = 0;
    const double *partY = nullptr;
    int nPartY = 0;
    int *eSlot = nullptr;    // block 0 records eX here (may be null)
    // non-null: the epilogue writes C's parts, row-major (prm) and
    // transposed (ptr), ld x ld, instead of C
    void *prm[3] = {}, *ptr[3] = {};
};

int split_parts(int mode);  // 16-bit parts per operand (0 for MPOW_FP32)
// BF16 modes: products write the next operand's parts in their epilogue
// (no separate split pass after each product).
inline bool split_fused(int mode) { return mode == MPOW_BF16X3 || mode == MPOW_BF16X6; }
int gemm_split_mode(int kernel);  // the mode of a split kernel id, -1 if none
int split_ld(int n);
hipError_t launch_split(int mode, const SplitLaunch &sl, hipStream_t s);
int gemm_split_pick(int mode, int n);
int gemm_split_tiles(int kernel, int n);
const char *gemm_split_name(int kernel);
hipError_t gemm_split_launch(int kernel, const SplitGemmLaunch &g, hipStream_t s);

// Float32 product kernel variants (index = MPOW_KERNEL_* id).
// Estimated rate of a tile shape for an n x n product: `rate`, its rate when
// every one of the 256 CUs runs whole waves of tiles, times the filled
// fraction of the last wave of workgroups, (T / 256) / ceil(T / 256) for T
// output tiles of bm x bn.
inline double tile_fill_rate(double rate, int n, int bm, int bn) {
    const double T = (double)((n + bm - 1) / bm) * (double)((n + bn - 1) / bn);
    const double waves = (double)(int64_t)((T + 255.0) / 256.0);
    return rate * (T / 256.0) / waves;
}
int gemm_pick(int n, bool vec4);            // default kernel id for size n
// The product kernel a power on workspace ws uses at size n: the forced
// kernel, else the tuned pick for n's bucket, else the per-size default
// (float32: gemm_pick, before gemm_resolve; split modes: gemm_split_pick).
int ws_product_kernel(const Workspace &ws, int n, bool vec4);
bool gemm_is_f32(int kernel);
int gemm_tiles(int kernel, int n);          // number of tiles (= partials written)
// The kernel id that runs for `kernel` at size n: the LDS-DMA kernels need
// 16-byte loads (vec4) and n <= 23170, else a same-order fallback runs.
int gemm_resolve(int kernel, int n, bool vec4);
const char *gemm_name(int kernel);
// axpi: the epilogue C = alpha X'Y' + I (matrix-exponential steps)
hipError_t gemm_launch(int kernel, const GemmLaunch &g, bool vec4, hipStream_t s, bool axpi = false);

// Scale and bookkeeping kernels.
int norm_blocks(int n);
hipError_t launch_sumsq(const float *A, int n, double *part, int blocks, hipStream_t s);
hipError_t launch_identity(float *out, int n, double *log2_scale, hipStream_t s);
hipError_t launch_finish(const float *C, int n, const double *partC, int nPartC,
                         const int *escale, int64_t p, float *out, double *log2_scale,
                         hipStream_t s, int naive_steps = -1);

// ---------------------------------------------------------------- ragged batch

// Descriptors the host fills (sorted by work), after a header holding the
// claim counter; per-worker scratch.
// A batch runs as up to kBatchGroups launches, one per kernel instance it
// needs; group g's descriptors are begin[g] .. end[g] - 1, claimed in order
// through counter[g] (the host copy resets the counters to 0).
constexpr int kBatchGroups = 5;
struct BatchHeader {
    int counter[kBatchGroups];
    int begin[kBatchGroups];
    int end[kBatchGroups];
    int count;
};
static_assert(sizeof(BatchHeader) % 16 == 0, "descriptors after the header stay 16-byte aligned");
struct BatchItem {
    const float *A;
    float *out;
    double *scale;  // null: no log2 scale for this matrix
    int64_t p;
    int n;
    int cfg;        // tile shape id (0: 128x128, 1: 64x64, 2: 256x256, 3-4: whole power)
};
struct BatchLaunch {
    void *desc;           // BatchHeader followed by the items
    float *scratch;       // grid * 2 * slot_floats floats
    int64_t slot_floats;  // floats per scratch buffer (max batched n squared)
    int group = 0;        // the descriptor group this launch works through
};
constexpr int kBatchMaxN = 256;
constexpr int kTileBuckets = kBatchMaxN / 16 + 1;  // bucket b holds n in (16(b-1), 16b]
// Tile shape ids: 0 = 128x128, 1 = 64x64, 2 = 256x256 (tiled products
// through per-worker scratch), 3 = the whole power in one workgroup with its
// operands resident in LDS where n <= 128 (streamed panels above), 4 = the
// whole power in one workgroup with streamed panels.
constexpr int kBatchShapes = 5;
// Kernel instances: 0: 64x64; 1: 128x128 + 64x64; 2: 256x256; 3: LDS-DMA
// 128/64; whole power per workgroup (power_wg.h): 4 resident n <= 64,
// 5 resident n <= 128, 6 panels n <= 256, 7 panels n <= 128
constexpr int kBatchInstances = 8;
// Instances that use the workers' scratch buffers (not the resident ones).
bool batched_uses_scratch(int inst);
// Workers whose scratch a context must hold: the largest grid of the
// instances that use scratch (launch groups run one after another).
int batch_scratch_workers(const int workers[kBatchInstances]);
int batched_cfg_for(int n);
// Resident workers per CU of kernel instance inst (0: 64x64 only, 1: 128x128
// and 64x64, 2: 256x256 and 128x128 with 8 waves).
int batched_occupancy(int inst);
hipError_t launch_batched(const BatchLaunch &b, int grid, int inst, hipStream_t s);
// Kernel instance for a batch: `need` = the smallest register-staged instance
// holding every tile shape used (0, 1 or 2); all_vec = every matrix allows
// 16-byte loads.
int batch_instance(int need, bool all_vec);

// One descriptor buffer of a batch context: device descriptors, the pinned
// host copy the descriptor copy reads, a captured graph (copy + launch) and
// the event recorded after the batch.
struct BatchSlot {
    void *desc = nullptr;
    void *host = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_count = -1;
    int graph_inst[kBatchGroups] = {-1, -1, -1, -1, -1};  // instance of each group's launch (-1: none)
    hipEvent_t done = nullptr;
    bool pending = false;
};

// Everything one stream of ragged batches needs.  Two descriptor slots are
// used alternately, so the host fills one while the batch of the other runs;
// both batches share the per-worker scratch, so a batch always waits (on the
// device) for the previous one.
struct BatchContext {
    BatchSlot slot[2];
    int next = 0;  // slot of the next batch
    int last = -1; // slot of the previous batch
    float *scratch = nullptr;
    int64_t slot_floats = 0;
    int workers[kBatchInstances] = {};  // grid of each kernel instance
    int max_batch = 0;
    int cfg[kTileBuckets] = {};
    hipStream_t capture_stream = nullptr;
};
size_t batch_desc_bytes(int max_batch);
// Device bytes (two descriptor buffers + scratch for `workers` workers).
size_t batch_device_bytes(int max_batch, int bmax, int workers);
// Sets up a context over [dev, dev + batch_device_bytes(..., max of
// workers)); creates the pinned buffers, capture stream and events.
hipError_t batch_context_init(BatchContext *bc, char *dev, int max_batch, int bmax,
                              const int workers[kBatchInstances]);
void batch_context_release(BatchContext *bc);
// Waits until every enqueued batch of the context has finished.
hipError_t batch_wait_all(BatchContext *bc);
// Fills descriptors in longest-work-first order and enqueues the batch on s
// (through the slot's captured graph when use_graph); returns the event that
// completes with the batch in *done (may be null).  scale may be null, or
// hold a per-item pointer that may itself be null.
hipError_t batch_enqueue(BatchContext *bc, int count, const float *const *A, const int *n,
                         const int64_t *p, float *const *out, double *const *scale,
                         hipStream_t s, bool use_graph, hipEvent_t *done = nullptr);

// Resident workers of each batched kernel instance on `device` (CUs x
// occupancy); false on failure.
bool batch_workers_for(int device, int workers[kBatchInstances]);

}  // namespace mpow

struct mpow_plan {
    int device = 0;
    int max_n = 0;
    int max_batch = 0;
    int mode = 0;
    uint32_t flags = 0;
    int last_error = 0;
    char *base = nullptr;  // the plan's single device allocation
    mpow::Workspace ws;
    mpow::TimingSink timing;
    mpow::BatchContext batch;
    float *expm_T = nullptr;    // Taylor polynomial of mpow_expm (MPOW_FLAG_EXPM)
    int *expm_e_dev = nullptr;  // norm exponent of its input, device
    int *expm_e_host = nullptr; // and its pinned host copy
};
