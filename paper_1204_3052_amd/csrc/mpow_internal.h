// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mpow.h"

namespace mpow {

// Workspace layout of one plan (all device memory, allocated at plan creation).
//  buf[0], buf[1]  ping-pong running matrices, max_n^2 floats each
//  part[0], part[1] per-tile partial sums of squares of buf[0] / buf[1]
//  partA            per-block partial sums of squares of the input A
//  escale           escale[k] = floor(log2 ||C_k||_F) of the k-th product's
//                   output (C_0 = A), written by the kernel that consumes C_k
struct Workspace {
    // split modes: hi/lo of the running matrix (row-major, transposed) and of A
    void *sx[4] = {nullptr, nullptr, nullptr, nullptr};
    void *sa[4] = {nullptr, nullptr, nullptr, nullptr};
    float *buf[2] = {nullptr, nullptr};
    double *part[2] = {nullptr, nullptr};
    double *partA = nullptr;
    int *escale = nullptr;
    size_t part_cap = 0;   // doubles in each part[] array
    size_t partA_cap = 0;  // doubles in partA
};

// How one product kernel is launched.
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
};

// Split of a float32 matrix into 16-bit hi/lo, row-major and transposed,
// zero-padded to ld x ld.
struct SplitLaunch {
    const float *X;
    const double *part;   // partial sums of squares of X
    int nPart;
    int n, ld;
    void *hi, *lo, *hiT, *loT;
    int *eSlot;           // block (0,0) records e of X here (may be null)
};

// Split-precision product: C = (X'Y') * 2^-2k from the hi/lo halves.
struct SplitGemmLaunch {
    const void *xh, *xl;  // left operand, row-major, ld
    const void *yh, *yl;  // right operand, transposed, ld
    float *C;
    double *partC;
    int n, ld;
};

int split_ld(int n);
hipError_t launch_split(int mode, const SplitLaunch &sl, hipStream_t s);
int gemm_split_pick(int mode, int n);
int gemm_split_tiles(int kernel, int n);
const char *gemm_split_name(int kernel);
hipError_t gemm_split_launch(int kernel, const SplitGemmLaunch &g, hipStream_t s);

// Ragged batch: descriptors the host fills (sorted by work), a header with
// the claim counter, and per-worker scratch.
struct BatchHeader {
    int counter;  // next descriptor to claim; the host copy resets it to 0
    int count;
    int pad[2];
};
struct BatchItem {
    const float *A;
    float *out;
    double *scale;  // null: no log2 scale for this matrix
    int64_t p;
    int n;
    int cfg;        // tile shape id (0: 128x128, 1: 64x64, 2: 128x64, 3: 64x128)
};
struct BatchLaunch {
    void *desc;           // BatchHeader followed by the items
    float *scratch;       // grid * 2 * slot_floats floats
    int64_t slot_floats;  // floats per scratch buffer (max batched n squared)
};
constexpr int kBatchMaxN = 256;
int batched_cfg_for(int n);
int batched_occupancy();  // resident workers per CU
hipError_t launch_batched(const BatchLaunch &b, int grid, hipStream_t s);

// Product kernel variants (index = MPOW_KERNEL_* id).
int gemm_pick(int n);                       // kernel id used for size n
int gemm_tiles(int kernel, int n);          // number of tiles (= partials written)
const char *gemm_name(int kernel);
hipError_t gemm_launch(int kernel, const GemmLaunch &g, bool vec4, hipStream_t s);

// Scale and bookkeeping kernels.
int norm_blocks(int n);
hipError_t launch_sumsq(const float *A, int n, double *part, int blocks, hipStream_t s);
hipError_t launch_identity(float *out, int n, double *log2_scale, hipStream_t s);
hipError_t launch_finish(const float *C, int n, const double *partC, int nPartC,
                         const int *escale, int64_t p, int steps, float *out,
                         double *log2_scale, hipStream_t s);

}  // namespace mpow

using mpow::kBatchMaxN;

struct TimingRecord {
    int kernel;
    double flop;
    hipEvent_t start, stop;
};

struct mpow_plan {
    int device = 0;
    int max_n = 0;
    int max_batch = 0;
    int mode = 0;
    uint32_t flags = 0;
    int last_error = 0;
    mpow::Workspace ws;
    // timing (MPOW_FLAG_TIMING)
    std::vector<hipEvent_t> free_events;
    std::vector<TimingRecord> pending;
    int64_t launches[MPOW_KERNEL_COUNT] = {};
    double ms[MPOW_KERNEL_COUNT] = {};
    double flop[MPOW_KERNEL_COUNT] = {};
    // ragged batch (max_batch > 0)
    void *batch_desc = nullptr;    // device: BatchHeader + max_batch items
    void *batch_host = nullptr;    // pinned host copy the graph's memcpy reads
    float *batch_scratch = nullptr;
    int64_t batch_slot_floats = 0;
    int batch_workers = 0;
    int batch_cfg[kBatchMaxN / 16 + 1] = {};  // tile shape per n bucket ((n+15)/16)
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_count = -1;
    hipEvent_t batch_done = nullptr;
    bool batch_pending = false;
};
