/*
 * givscore -- least-squares scores of every family (child, parent set) of m
 * variables by a walk over QR decompositions with Givens retriangularisations.
 *
 * The method (Alipourfard & Gao, "Solving All Regression Models For Learning
 * Gaussian Networks Using Givens Rotations"):
 *   - one QR decomposition of the n x m data matrix X (Sec. 2: the algorithm
 *     starts from the QRD of the data);
 *   - a sequence of adjacent column transpositions, each followed by one Givens
 *     rotation that restores the triangular R (Sec. 1.3, the GRC operator);
 *   - every R visited solves the regressions "prefix -> later variable" of its
 *     column ordering (Sec. 2); the sequence is the shortest one that visits every
 *     parent set (Sec. 3 recursion, Sec. 4 optimality), split into independent
 *     pieces that start from their own QRD (Sec. 6).
 *
 * Family set and table layout (the paper leaves both implicit):
 *   families: child c in 0..m-1, parent set S any subset of the other m-1
 *             variables, the empty set included: m * 2^(m-1) families (Sec. 1).
 *   index(c, S) = c * 2^(m-1) + compress(S, c), where compress removes bit c of
 *             the bitmask S (bit v = variable / column v) and shifts the higher
 *             bits down by one.  gs_family_index() computes it.
 *   RSS(c, S) = min_beta || x_c - X_S beta ||^2  (no intercept; X used as given).
 *   BIC(c, S) = n ln(RSS / n) + (|S| + 2) ln n   (lower is better).
 *
 * Conventions for every entry point:
 *   - Return value: GS_OK (0) or a negative gs_status.  Argument errors are found
 *     before any device work and leave every output untouched.  gs_last_error()
 *     gives a message for the calling thread's last failure.
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The caller owns every pointer it passes.
 *     The library owns the plan and its device workspace; gs_plan_destroy frees them.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream).  Device
 *     work is enqueued asynchronously on it; outputs are valid once the stream has
 *     reached that point.  Data-dependent conditions found on the device (rank
 *     deficiency, non-finite input) are reported by gs_sync_status().
 *   - A plan may be used by one stream at a time (its workspace is shared).
 */
#ifndef GIVSCORE_H
#define GIVSCORE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gs_plan_s gs_plan_t;

typedef enum {
    GS_OK = 0,
    GS_EINVAL = -1,      /* bad argument: null pointer, size or range            */
    GS_ERANK = -2,       /* X is numerically rank deficient: some column lies
                            within an angle of n*eps of the span of the others    */
    GS_ENOMEM = -3,      /* device workspace could not be allocated               */
    GS_EHIP = -4,        /* a HIP runtime call failed                             */
    GS_ENOTFINITE = -5,  /* X holds NaN or Inf                                    */
    GS_ERANGE = -6       /* RSS output only: some RSS lies outside the normal range
                            of the table's type (written as inf, or as a subnormal
                            or zero that lost relative precision)                 */
} gs_status;

typedef enum { GS_OUT_BIC = 0, GS_OUT_RSS = 1 } gs_output;

/* Largest number of variables supported (the FP32 table then takes 64 GB). */
#define GS_MAX_M 30

typedef struct {
    int m;                      /* variables                                          */
    int k;                      /* variables walked inside one segment (Sec. 6: m - k
                                   variables are fixed in front or at the back)       */
    int ks;                     /* inner block: the lowest ks labels, walked by the
                                   paper's sequence for ks variables                  */
    int q;                      /* k - ks middle variables, walked by the same
                                   sequence one level up                              */
    int64_t num_segments;       /* 2^(m-k) independent segments                       */
    int64_t sub_per_segment;    /* 2^q inner walks per segment                        */
    int64_t swaps_per_segment;  /* Givens steps per segment: 2^k - k - 1              */
    int64_t num_families;       /* m * 2^(m-1)                                        */
    int64_t num_waves;          /* 64-lane waves the segments are packed into         */
} gs_plan_info_t;

/* Number of families m * 2^(m-1) (Sec. 1: every child with every subset of the other
 * m - 1 variables, the empty set included); -1 if m is outside 1..GS_MAX_M. */
int64_t gs_num_families(int m);

/* Table index of (child, parent_mask) in the layout above (the paper's score table of
 * Sec. 1 and Sec. 3 has no stated order; this is the library's); -1 if child is out of
 * range, bit `child` is set in parent_mask, or parent_mask has bits at or above m. */
int64_t gs_family_index(int m, int child, uint64_t parent_mask);

/* The paper's swap sequence Upsilon(m) (Sec. 3 recursion with the "+1" shift,
 * Sec. 5 recurrence): 1-based indices i, each exchanging positions i and i+1.
 * Writes min(cap, 2^m - m - 1) entries to out (host) and returns the full length,
 * or GS_EINVAL for m outside 1..24. */
int64_t gs_upsilon(int m, int32_t *out, int64_t cap);

/* Create a plan for m variables (1..GS_MAX_M) with the default segment sizes: the
 * split of Sec. 6 / Alg. 2 into 2^(m-k) independent segments, each walking k
 * variables along Upsilon(k) (Sec. 3) with the other m - k fixed in front or behind,
 * packed into 64-lane waves.  Host-only integer work; no device memory is touched
 * until the first score call.  *out receives a library-owned handle. */
int gs_plan(int m, gs_plan_t **out);

/* Same with explicit sizes (Sec. 6: k walked variables per segment; ks the inner
 * block walked by Upsilon(ks) at every resting point of the middle variables):
 * 1 <= ks <= 6, ks <= m, ks <= k <= m, k - ks <= 16.  ks = 0 or k = 0 selects the
 * default for that size.  Lanes per segment and waves per CU are not parameters: a
 * segment takes one lane per column it walks or carries (k + its back variables),
 * segments are packed side by side into 64-lane waves, and the kernels' register and
 * LDS budgets fix the waves per CU (4 per SIMD for the FP32 walk with ks = 5). */
int gs_plan_tuned(int m, int k, int ks, gs_plan_t **out);

/* Free a plan and its device workspace (NULL is ignored); waits for the plan's last
 * enqueued work. */
void gs_plan_destroy(gs_plan_t *plan);

/* Device bytes the plan's workspace takes for data of n rows (backward != 0: including
 * the adjoint's buffers), host integer arithmetic only.  Setting the environment
 * variable GS_WORKSPACE_LIMIT to a byte count makes every call whose workspace would
 * exceed it fail with GS_ENOMEM before touching the device. */
int gs_plan_workspace_bytes(const gs_plan_t *plan, int64_t n, int backward, int64_t *bytes);

/* Sizes chosen by the plan (host struct; Sec. 6 segment split, Sec. 3 sequence
 * lengths). */
int gs_plan_get_info(const gs_plan_t *plan, gs_plan_info_t *info);

/* Host simulation of the plan's walk: counts[index] += 1 for every family the
 * kernels will write (counts: host, len >= m * 2^(m-1)).  The split of Sec. 6 covers
 * every family exactly once, so a correct plan leaves every entry at 1.  For testing
 * the planner; m <= 22 (gs_count_writes checks the kernels at any size). */
int gs_plan_count_emissions(const gs_plan_t *plan, int32_t *counts, int64_t len);

/* R0 = the triangular factor of the QR decomposition of X (Sec. 2, the initial
 * QRD), FP64, with a non-negative diagonal.
 *   X: device, n x m, row-major, row stride ldx >= m (elements), n > m.
 *   R0: device, m x m row-major; the strict lower triangle is set to zero. */
int gs_qr_r0(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
             double *R0, void *stream);

/* Scores of all m * 2^(m-1) families (Sec. 1) by the walk: one QRD of X (Sec. 2),
 * then the shortest sequence of adjacent column swaps, each retriangularised by one
 * Givens rotation (Sec. 1.3, Sec. 3-4), every visited R read out as the RSS of its
 * prefix regressions (Sec. 2), split into independent segments (Sec. 6).  The walk
 * runs in FP32; R0 and each segment's starting R are FP64.
 *   X: device, n x m row-major FP64, row stride ldx >= m, n > m; m must equal the
 *      plan's m.
 *   scores: device, m * 2^(m-1) floats, 16-byte aligned, written in table order
 *      (every entry exactly once).
 *   what: GS_OUT_BIC or GS_OUT_RSS. */
int gs_score_all(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                 float *scores, int what, void *stream);

/* Fused consumer of the scores: score-based learning uses the local scores of all
 * families (Sec. 1), most often as the best parent set per child, a short list of the
 * best ones, or a soft minimum over all of them.  gs_score_reduce runs the FP32 BIC
 * walk of gs_score_all but folds every value into per-child results on chip instead of
 * writing the m 2^(m-1) table (the paper keeps O(m^2) working storage, Sec. 7; here a
 * few floats per child and segment).  Per child c (arrays of m, device memory):
 *   best_score[c]    min over parent sets S of BIC(c, S);
 *   best_parents[c]  a parent mask S reaching it (bit v = variable v; the smallest mask
 *                    among equal values);
 *   logsumexp[c]     ln sum over S of exp(-BIC(c, S)), accumulated relative to the
 *                    minimum (double);
 *   top_score[c * top_k + j], top_parents[...]: the top_k (0..8) smallest BIC values of
 *                    child c, ascending, with their parent masks (may be NULL if
 *                    top_k = 0).
 * BIC values are those gs_score_all writes (same kernels, same arithmetic).  The merge
 * over segments runs in a fixed order: the results are reproducible bit for bit.
 * Workspace: about m 2^(m-k) x 76 bytes beyond gs_score_all's, allocated on the first
 * call. */
#define GS_REDUCE_MAX_TOPK 8
typedef struct {
    float *best_score;
    uint32_t *best_parents;
    double *logsumexp;
    float *top_score;
    uint32_t *top_parents;
    int top_k;
} gs_reduce_t;
int gs_score_reduce(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                    const gs_reduce_t *out, void *stream);

/* gs_score_all without allocation, for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, kernels and results as gs_score_all (bit for bit), but every piece
 * of workspace lives in a file-scope device array of GS_STATIC_SCRATCH_BYTES
 * (32 MiB), which each device that runs this call holds until the process ends; no
 * allocation of any kind happens in the call.  The plan's walk program and lane
 * tables are copied into that array (hipMemcpyAsync from the plan's host memory on
 * `stream`) when the previous call on the device used another plan.
 *   status_code: device int (or NULL); receives the gs_status of the data (GS_OK,
 *     GS_ERANK, GS_ENOTFINITE, GS_ERANGE) when the stream reaches the end of the call
 *     (the plan's gs_sync_status does not see this path).
 * Returns GS_ENOMEM, before any device work, when the plan and n need more than the
 * array holds (m = 26 with the default plan needs about 16 MB at n = 5000; m >= 28
 * does not fit).  All calls on one device share the array and it keeps the last
 * call's contents: calls that overlap on a device race and must be serialised by the
 * caller. */
#define GS_STATIC_SCRATCH_BYTES (32u << 20)
int gs_score_all_static(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                        float *scores, int what, int *status_code, void *stream);

/* Many datasets of one shape, each scored as by gs_score_all (FP32 walk), with up to
 * in_flight of them in progress at once.  Every dataset is its own instance of the
 * problem of Sec. 1; its work splits into independent pieces (Sec. 6), and pieces of
 * different datasets can run side by side like those of one: here one dataset's R0 and
 * anchors overlap another's walk, and the walks share the device.  The plan keeps
 * in_flight - 1 extra workspaces (plans with its m, k and inner block) and in_flight
 * internal streams, created on the first call that needs them; the streams fork from
 * `stream` and `stream` waits for all of them before its later work.
 *   X[i]: device, n x m row-major FP64 (row stride ldx), i = 0..count-1;
 *   scores[i]: device, m * 2^(m-1) floats, 16-byte aligned (table order of
 *     gs_family_index); every table is bit-identical to gs_score_all on X[i] alone;
 *   what: GS_OUT_BIC or GS_OUT_RSS; in_flight: 1..GS_MANY_MAX_IN_FLIGHT.
 * The arrays X and scores are host arrays of device pointers, read during the call.
 * gs_many_status gives each dataset's status (gs_sync_status does not cover this call).
 * As for every call on a plan, calls that overlap on one plan race (the slots are the
 * plan's).  Errors: GS_EINVAL on bad arguments (before any device work), GS_ENOMEM; an
 * error after some datasets were enqueued still makes `stream` wait for them. */
#define GS_MANY_MAX_IN_FLIGHT 8
int gs_score_all_many(gs_plan_t *plan, int count, const double *const *X, int64_t n,
                      int64_t ldx, float *const *scores, int what, int in_flight, void *stream);

/* Per-dataset status of the last gs_score_all_many call on this plan: waits for it,
 * writes count codes (GS_OK, GS_ERANK, GS_ENOTFINITE, GS_ERANGE) to status (host) and
 * returns the first non-OK code in dataset order (GS_OK if none).  GS_EINVAL if the
 * plan has not run gs_score_all_many. */
int gs_many_status(gs_plan_t *plan, int *status);

/* Testing: the FP32 walk of gs_score_all (same plan, same launch, same store path)
 * with every table write replaced by an atomic increment of a 32-bit counter at the
 * same index: counts (device, m * 2^(m-1) uint32, 16-byte aligned, zeroed by the
 * caller) receives +1 per write.  The paper's split (Sec. 6, Alg. 2) covers every
 * family exactly once, so a correct plan and kernel leave every counter at 1. */
int gs_count_writes(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                    uint32_t *counts, void *stream);

/* Regression coefficients of every family: Sec. 1.1 solves a regression from its QRD
 * by back-substitution, O(|S|^2), and every R the walk visits is the QRD of its column
 * ordering, so each family takes its coefficients from the R that solves it (Sec. 2):
 * R[P][P] beta = R[P][c] for the prefix P.  FP64 walk over segments of up to 10
 * variables (Sec. 6 split), R0 and segment starts as for the scores.
 *   beta: device, m * 2^(m-1) rows of m doubles, row index(c, S) (table order): beta_v
 *     for v in S, zeros elsewhere (the child included), so x_c - X beta_row is the
 *     residual whose squared norm is RSS(c, S).  16-byte aligned; 8 m^2 2^(m-1) bytes
 *     (1.7 GB at m = 20), hence m <= GS_BETA_MAX_M.
 * The plan's m must equal m (its segment sizes are not used). */
#define GS_BETA_MAX_M 22
int gs_score_beta(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                  double *beta, void *stream);

/* Same method with the whole walk in FP64 and an FP64 table (16-byte aligned). */
int gs_score_all_f64(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                     double *scores, int what, void *stream);

/* Reverse mode of gs_score_all: given dscores = d(loss)/d(score) for every family
 * (table order; the score is BIC or RSS as selected by `what`), writes
 * dX = d(loss)/dX.  Not in the paper: the adjoint of its method.
 *   X: device, the same n x m FP64 data as for gs_score_all (row stride ldx).
 *   dscores: device, m * 2^(m-1) floats, 16-byte aligned (GS_EINVAL otherwise).
 *   dX: device, n x m FP64, row stride lddx >= m; overwritten.
 * The FP32 walk is replayed and then undone step by step in FP32: every Givens step
 * is recovered from the rotated matrix, nothing is stored per step.  The reverse
 * rules of the segment-anchor QRs and of R0 are applied in FP64; all sums run in a
 * fixed order, so the result is reproducible bit for bit.  Workspace: about
 * 2^(m-k) (k + m^2/32 + 1) x 256 bytes, plus 2^(m-k) k x 256 bytes for segments of
 * k >= 9 (whose reverse walk starts from anchors formed in the walk's final ordering
 * instead of a replay), allocated on the first call. */
int gs_score_backward(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                      const float *dscores, int what, double *dX, int64_t lddx, void *stream);

/* Same with the walk replayed and undone in FP64 and FP64 dscores (16-byte aligned). */
int gs_score_backward_f64(gs_plan_t *plan, const double *X, int64_t n, int m, int64_t ldx,
                          const double *dscores, int what, double *dX, int64_t lddx,
                          void *stream);

/* Reuse of the forward's intermediates by the backward (off by default).  With
 * enable != 0, gs_score_backward (gs_score_backward_f64) takes R0 and the segment
 * anchors from the plan's buffers instead of forming them again when the plan's last
 * call that formed them (gs_score_all, gs_score_reduce, gs_count_writes or a backward
 * call for the FP32 walk; gs_score_all_f64 or gs_score_backward_f64 for the FP64 walk)
 * was given the same X pointer, n and ldx, and no call since has rewritten R0
 * (gs_qr_r0, gs_score_beta); otherwise it forms them as usual.  The caller guarantees
 * that X still holds the same values as in that call.  The status word is then the
 * one that call left.  Returns GS_OK, or GS_EINVAL for a NULL plan. */
int gs_plan_set_reuse(gs_plan_t *plan, int enable);

/* Wait for the plan's last enqueued work and return GS_OK, GS_ERANK, GS_ENOTFINITE
 * or GS_ERANGE from the device status word of that call (GS_EHIP on a runtime
 * failure). */
int gs_sync_status(gs_plan_t *plan);

/* Variance inflation factors of the data of the plan's last call, computed from
 * its R0: vif[c] = ||x_c||^2 [(X^T X)^-1]_cc = ||x_c||^2 / RSS(c | all other
 * columns), c = 0..m-1 (host array of m doubles; inf for a singular X).  Waits for
 * that call.  They bound the sensitivity of every RSS to rounding (no residual of x_c
 * is smaller than ||x_c||^2 / vif[c]) and so state how far the FP32 walk can be
 * trusted on this data; the walks are scale free (the columns are equilibrated by
 * powers of two), so the units of X do not matter.  Not in the paper: its scores are
 * exact arithmetic. */
int gs_column_vif(gs_plan_t *plan, double *vif);

/* Measurement: per-stage timing with HIP events recorded on the call's stream.
 * enable != 0 starts recording (and clears old records). */
int gs_set_timing(gs_plan_t *plan, int enable);

/* Waits for the recorded events and returns, for the calls recorded since the last
 * gs_set_timing, the mean milliseconds of: ms[0] R0 QR, ms[1] segment anchors,
 * ms[2] walk kernel, ms[3] whole call (host arrays of 4).  *count = calls averaged. */
int gs_get_timing(gs_plan_t *plan, double *ms, int64_t *count);

/* ---- Batched scoring: many datasets, one launch per stage -------------------
 * Sec. 6 splits one walk over processors; a batch runs the walks of many datasets
 * of different m and n (e.g. bootstrap resamples) side by side: one TSQR launch per
 * pass over all row blocks of all datasets, one anchor launch over all segments, one
 * walk launch over all packed waves (longest walk first).  FP32 walk, inner blocks
 * of 5 variables.  The sequence can be captured once into a hipGraph and replayed. */
typedef struct gs_batch_s gs_batch_t;

typedef struct {
    const double *X;  /* device, n x m row-major FP64 (the sizes given at creation) */
    int64_t ldx;      /* row stride of X, >= m                                       */
    float *scores;    /* device, m * 2^(m-1) floats, 16-byte aligned, table order    */
} gs_batch_data_t;

/* Plan a batch of `count` (1..4096) datasets: m[i] in 5..GS_MAX_M, n[i] > m[i]
 * (host arrays).  k (host array or NULL) selects each dataset's segment size as in
 * gs_plan_tuned (0 = default).  Host-only work; device memory is allocated on the
 * first gs_score_batched call. */
int gs_batch_create(int count, const int *m, const int64_t *n, const int *k, gs_batch_t **out);

/* Free a batch, its device workspace and its graphs (NULL is ignored); waits for
 * the batch's last enqueued work. */
void gs_batch_destroy(gs_batch_t *batch);

/* Total packed waves, segments and families of the batch (host outputs, each may be
 * NULL). */
int gs_batch_info(const gs_batch_t *batch, int64_t *total_waves, int64_t *total_segments,
                  int64_t *total_families);

/* Scores of every family of every dataset.  data: host array of `count` entries.
 * what: GS_OUT_BIC or GS_OUT_RSS.  use_graph != 0 replays a hipGraph captured on the
 * first such call for this `what` (the kernels read the data pointers from a device
 * table, so a call with different pointers only rewrites the table, after waiting for
 * the batch's previous call).  Calls on one batch must not overlap. */
int gs_score_batched(gs_batch_t *batch, const gs_batch_data_t *data, int what, int use_graph,
                     void *stream);

/* Wait for the batch's last call; status[i] (host, count entries) gets GS_OK,
 * GS_ERANK or GS_ENOTFINITE for dataset i.  Returns GS_OK or the status of a failed
 * dataset. */
int gs_batch_status(gs_batch_t *batch, int *status);

/* Message for the calling thread's last error ("" if none). */
const char *gs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GIVSCORE_H */
