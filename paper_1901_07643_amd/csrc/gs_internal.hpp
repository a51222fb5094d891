// Internal declarations of libgivscore: the plan object and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/givscore.h"
#include "walk_program.hpp"

// Device status word bits (OR-ed by kernels).
#define GS_FLAG_NOTFINITE 1
#define GS_FLAG_RANK 2
#define GS_FLAG_GUARD 4  // a Givens pivot pair may be (near) zero: take the guarded steps
#define GS_FLAG_RANGE 8  // an RSS value left the output type's normal range

// Column statistics of one dataset.  Before the QR, X is scaled by powers of two
// so that every column's largest magnitude lies in [1/2, 1) (exp0: the column
// maxima's exponents, INT_MIN until the first block reports); the TSQR then works on
// X 2^-exp0, whose squares stay inside the double range, and the stored R0 is the R of
// that matrix.  The last TSQR pass derives the walk's equilibration: scale[c] turns
// column c of the stored R0 into a column of norm in [1/2, 1), and X D, D =
// diag(2^-exp2), is the matrix the walk scores.  RSS(c, S) of X is RSS of X D times
// 2^(2 exp2[c]) (scaling a parent does not change a residual).
struct ColStats {
    double scale[32];  // column scale of the stored R0 (a power of two)
    double vif[32];    // variance inflation factor ||x_c||^2 [(X^T X)^-1]_cc (inf if singular)
    int exp2[32];      // X D = X 2^-exp2
    int exp0[32];      // pre-scaling of X before the QR
};
// A VIF above this (an angle below 1e-4 rad between a column and the span of the
// others) makes the walks take the guarded Givens steps.
constexpr double GS_GUARD_VIF = 1e8;


// Per (child, segment) partial results of the fused reduction (index child * nseg +
// segment): the minimum BIC, its parent set, the sum of exp(min - BIC) over the
// segment's parent sets, and (top-k mode) the GS_REDUCE_TOPK smallest values, ascending.
#define GS_REDUCE_TOPK 8
// The child merge runs in two launches: up to GS_REDUCE_SPLIT workgroups per child
// reduce fixed slices of the segments into a ReduceStage each, then one wave per
// child merges those in order.
#define GS_REDUCE_SPLIT 32
struct ReduceStage {
    double mn, sum;
    uint32_t mask;
    float tv[GS_REDUCE_TOPK];
    uint32_t tm[GS_REDUCE_TOPK];
};
struct ReducePartials {
    float *pmin = nullptr;
    uint32_t *pmask = nullptr;
    float *psum = nullptr;
    float *ptopv = nullptr;
    uint32_t *ptopm = nullptr;
    ReduceStage *stage = nullptr;  // m x GS_REDUCE_SPLIT
};

// The walk's state after its last sub-walk, the same for every segment: position r of
// the walked block holds variable order[r], and the inner block starts at middle row z.
struct WalkEnd {
    int8_t order[32];
    int z;
};

// The adjoint starts the reverse walk from anchors formed in the final ordering (one QR
// per segment) instead of replaying the walk, for segments of at least this many walked
// variables (shorter walks replay faster than the extra QR launch).
constexpr int ADJ_END_MIN_K = 9;

struct gs_plan_s {
    uint64_t id = 0;  // unique per plan created in this process
    int m = 0, k = 0, ks = 0, q = 0;
    int64_t nseg = 0, nsub = 0;
    std::vector<uint32_t> prog;  // 2 words per sub-walk (layout in walk_program.hpp)
    WalkEnd end{};               // the walk's state after the last sub-walk
    // segments packed into 64-lane waves: for wave w and lane x, lane_seg[64 w + x] is
    // the segment code (or -1) and lane_loc[64 w + x] the column slot inside it
    int64_t nwaves = 0;
    std::vector<int32_t> lane_seg;
    std::vector<int8_t> lane_loc;

    // device workspace, allocated on first use on `device`
    int device = -1;
    uint32_t *d_prog = nullptr;
    int32_t *d_lane_seg = nullptr;
    int8_t *d_lane_loc = nullptr;
    double *d_r0 = nullptr;      // m x m
    ColStats *d_stats = nullptr;  // column statistics of the last call's data
    double *d_qr_a = nullptr;    // TSQR ping-pong buffers
    double *d_qr_b = nullptr;
    int64_t qr_cap = 0;          // elements per TSQR buffer
    void *d_anchor = nullptr;    // nseg x k x 32 (float or double)
    void *d_tail = nullptr;      // nseg x 32
    int *d_status = nullptr;
    // adjoint workspace (allocated on the first backward call); d_anchor_end: anchors in
    // the walk's final ordering (k >= ADJ_END_MIN_K only)
    void *d_anchor_end = nullptr;
    double *d_anchorbar = nullptr;  // nseg x k x 32
    double *d_tailbar = nullptr;    // nseg x 32
    double *d_vout = nullptr;       // nseg x m x m
    double *d_partial = nullptr;    // chunks x m x m
    double *d_B = nullptr;          // m x m
    double *d_K = nullptr;          // m x m
    // fused-reduction partials (allocated on the first gs_score_reduce call)
    ReducePartials red;
    // coefficient walk: Upsilon(beta_k) on the device (first gs_score_beta call)
    int8_t *d_ups = nullptr;
    int beta_k = 0;
    hipStream_t last_stream = nullptr;
    hipEvent_t done = nullptr;
    // The data whose R0 and segment anchors the plan's buffers hold: set when a front half
    // has been enqueued in full, cleared by any call that rewrites R0.  With reuse_front
    // the backward entry points take them from there instead of forming them again.
    const void *front_x = nullptr;
    int64_t front_n = 0, front_ldx = 0;
    int front_elem = 0;  // bytes per anchor entry: 4 (FP32 walk) or 8 (FP64 walk)
    bool reuse_front = false;
    // gs_score_all_many: the extra in-flight workspaces (plans with the same program),
    // one stream and join event per slot, the fork event and per-dataset status words
    std::vector<gs_plan_s *> slots;
    std::vector<hipStream_t> slot_streams;
    std::vector<hipEvent_t> slot_join;
    hipEvent_t fork = nullptr;
    int *d_many_status = nullptr;
    int64_t many_cap = 0, many_count = 0;

    bool timing = false;
    std::vector<std::array<hipEvent_t, 4>> events;
};

namespace gs {

#ifdef __HIPCC__
// Order the LDS accesses of one wave: some lanes write, others read.  Without the
// fences the compiler may treat the cross-lane exchange as a data race and move
// the reads ahead of the writes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP64 1/sqrt(x) and 1/d from the hardware approximations, each refined by two Newton
// steps (about one ulp; the library's correctly rounded forms cost twice as many
// instructions).  For normal, finite arguments only.
__device__ __forceinline__ double rsq_newton(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return y;
}
__device__ __forceinline__ double rcp_newton(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}
constexpr double GS_DBL_MIN = 2.2250738585072014e-308;
#endif  // __HIPCC__: the host-only planner build sees none of the device helpers

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Host planner (plan.cpp)
int build_program(gs_plan_s *p);
// Upsilon(q) with 0-based swap positions (the paper's sequence minus one).
void upsilon0(int q, std::vector<int> &seq);

// One workgroup of a batched TSQR pass: rows [128 block, 128 block + 128) of A.
struct TsqrJob {
    const double *A;
    int64_t nrows;
    int64_t lda;
    double *Rout;  // m x m output of this block
    int *status;
    ColStats *stats;  // the dataset's statistics (pre-scaling read by pass 0, written last)
    int64_t n_orig;
    int m;
    int block;
    int first;    // pass 0: reads X, scales each column of the block by its own power of two
    int rescale;  // pass 1: brings the pass-0 blocks to the common scale
    int *eblk;    // the dataset's pass-0 block exponents (32 ints per block)
    int final_pass;
};

// One dataset of a batched call (device-side descriptor).  The walk of a batch
// always uses inner blocks of 5 variables (every dataset has m >= 5).
struct BatchItem {
    const double *R0;
    const ColStats *stats;
    const void *anchor;  // nseg x k x 32 (float)
    const void *tail;    // nseg x 32
    const uint32_t *prog;
    const int32_t *lane_seg;
    const int8_t *lane_loc;
    const int *status;
    void *out;  // the dataset's score table
    int m, k, ks, q;
    int64_t nseg, nsub, nwaves;
    double row_scale, nlog, lnn, nln2;
};
constexpr int BATCH_KS = 5;

// Kernel launchers (return hipError_t of the launch)
// TSQR of X (n x m, row stride ldx) into R0 (m x m, upper, non-negative diagonal).
// R0 of X 2^-exp0 goes to R0; with Rtrue != nullptr also the R factor of X itself.
// The status word and stats->exp0 must have been reset (launch_front_reset).
hipError_t launch_qr_r0(const double *X, int64_t n, int m, int64_t ldx, double *R0, double *Rtrue,
                        double *bufA, double *bufB, int *status, ColStats *stats, hipStream_t s);
// Reset the status words and the pre-scaling exponents of `count` datasets.
hipError_t launch_front_reset(int *status, ColStats *stats, int count, hipStream_t s);
int64_t qr_workspace_elems(int64_t n, int m);
int tsqr_rows_per_block();
hipError_t launch_tsqr_batched(const TsqrJob *jobs, int njobs, int mmax, hipStream_t s);

// Host planner: pack segments into 64-lane waves (plan.cpp).
int pack_waves(gs_plan_s *p);

// Segment anchors: R blocks of every segment from R0, computed in FP64 and stored
// as T (float for the FP32 walk, double for the FP64 walk).
template <typename T>
hipError_t launch_anchors(const double *R0, const ColStats *stats, int m, int k, int ks,
                          int64_t nseg, T *anchor, T *tail, hipStream_t s);
// The same rows of every segment with its walked block in the final ordering of the
// walk (end), in the row layout of that state; the tails are those of the start.
template <typename T>
hipError_t launch_anchors_end(const double *R0, const ColStats *stats, int m, int k, int ks,
                              int64_t nseg, const WalkEnd &end, T *anchor, hipStream_t s);

// Device tables a walk launch reads besides its anchors: the plan's program and packed
// lane tables, the dataset's status word and column statistics.
struct WalkTables {
    const uint32_t *prog;
    const int32_t *lane_seg;
    const int8_t *lane_loc;
    int *status;
    const ColStats *stats;
};

// The walk.  T = float or double; writes the full table.
hipError_t launch_walk_f32_tables(const gs_plan_s *p, const WalkTables &t, const float *anchor,
                                  const float *tail, float *out, int64_t n, bool bic,
                                  hipStream_t s);
hipError_t launch_walk_f32(const gs_plan_s *p, const float *anchor, const float *tail, float *out,
                           int64_t n, bool bic, hipStream_t s);
hipError_t launch_walk_f64(const gs_plan_s *p, const double *anchor, const double *tail,
                           double *out, int64_t n, bool bic, hipStream_t s);
// The FP32 BIC walk folding its values into per (child, segment) partials instead of
// writing the table (top: also the smallest GS_REDUCE_TOPK), then the per-child merge.
hipError_t launch_walk_reduce(const gs_plan_s *p, const float *anchor, const float *tail,
                              const ReducePartials &red, bool top, int64_t n, hipStream_t s);
hipError_t launch_reduce_children(const gs_plan_s *p, const ReducePartials &red, bool top,
                                  float *best, uint32_t *best_mask, double *lse, float *top_v,
                                  uint32_t *top_m, int top_k, hipStream_t s);
// Coefficients of every family by an FP64 walk over segments of k variables (ups:
// Upsilon(k), 0-based), out: m * 2^(m-1) rows of m doubles.
hipError_t launch_beta_walk(const double *R0, const ColStats *stats, int m, int k,
                            const int8_t *ups, int64_t nups, double *out, hipStream_t s);
// The FP32 walk with every table write replaced by an atomic +1 of a uint32 counter.
hipError_t launch_walk_count(const gs_plan_s *p, const float *anchor, const float *tail,
                             uint32_t *counts, int64_t n, hipStream_t s);

// Batched launches (one per stage for every dataset of a batch)
hipError_t launch_walk_batched_f32(const BatchItem *items, const int32_t *wave_item,
                                   const int32_t *wave_local, int64_t total_waves, int qmax,
                                   bool bic, hipStream_t s);
hipError_t launch_anchors_batched_f32(const BatchItem *items, const int64_t *seg_prefix, int count,
                                      int64_t total_segs, int mmax, hipStream_t s);

// Adjoint (adjoint.hip)
// anchor_end: anchors of the walk's final state (launch_anchors_end), from which the
// reverse walk starts; nullptr: the walk is replayed from `anchor` first.
template <typename T>
hipError_t launch_walk_adjoint(const gs_plan_s *p, const T *anchor, const T *tail,
                               const T *anchor_end, const T *dscores, double *anchorbar,
                               double *tailbar, int64_t n, bool bic, hipStream_t s);
int64_t adjoint_partial_chunks(int64_t nseg);
hipError_t launch_qr_adjoint_chain(const gs_plan_s *p, const double *R0, const ColStats *stats,
                                   bool bic, const double *anchorbar,
                                   const double *tailbar, double *vout, double *partial, double *B,
                                   double *K, const double *X, int64_t n, int64_t ldx, double *dX,
                                   int64_t lddx, hipStream_t s);

}  // namespace gs
