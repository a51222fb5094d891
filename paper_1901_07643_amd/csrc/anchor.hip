// Segment anchors: the R factor each segment's walk starts from (FP64).
//
// Sec. 6 gives every processor its own initial QRD but not how to form it.  A
// segment's ordering is [front variables, middle block, inner block, back
// variables]; since X P = Q0 (R0 P), the R of that ordering equals (up to row
// signs) the R of QR(R0 P), an m x m Householder QR instead of an n x m one.  The
// columns are equilibrated first (R0 D, D the power-of-two scales of the R0 pass):
// the walk then scores X D, whose residual sums differ from those of X only by the
// exact factor 2^(2 exp2[c]) of the child.
// Rows of the front variables never change during the walk and are dropped;
// rows of the back variables never change either and only enter through their
// squared sums (the "tail" of each back column).  Those sums are the same before
// and after the reflections of the back columns, so the QR stops after the front
// and walked columns: d + k of the m Householder steps.
//
// One 32-lane half-wave per segment; lane c holds column c of R0 P in registers
// (rows 0..MM-1, MM >= m).  Each Householder step broadcasts the pivot column
// through LDS and updates every column at once; the rows are then signed so that
// the diagonal is non-negative (the walk keeps it so, which lets its adjoint
// recover every rotation from the rotated matrix).
//
// Output layout, per segment s, by column slot l (l < k: variable l; l = k + i:
// the i-th back variable in ascending label order):
//   anchor[s][r][l], r = 0..k-1 the rows of the walked block by position (in the
//                    starting ordering the q middle rows, then the ks inner rows; in the
//                    final ordering of the walk, the middle rows in front of the inner
//                    block, its ks rows, then the middle rows behind it), l = 0..31
//   tail[s][l]     = sum of squares of column l over the back rows.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gs_internal.hpp"
#include "segment_qr.hpp"

namespace gs {

constexpr int ANCHOR_HALVES = 8;  // segments per 256-thread workgroup

// use_end: the walked block (positions d .. d+k-1) in the walk's final ordering end.order
// instead of the starting one; tail == nullptr: no tails written (they do not change
// along the walk).
template <int MM, typename TO>
__global__ __launch_bounds__(256) void anchor_kernel(const double *__restrict__ R0,
                                                     const ColStats *__restrict__ stats, int m,
                                                     int k, int ks, int64_t nseg,
                                                     TO *__restrict__ anchor,
                                                     TO *__restrict__ tail, WalkEnd end,
                                                     int use_end) {
    __shared__ double piv_col[ANCHOR_HALVES][MM];
    const int hw = threadIdx.x >> 5;
    const int c = threadIdx.x & 31;
    const int64_t seg = int64_t(blockIdx.x) * ANCHOR_HALVES + hw;
    const bool ok = seg < nseg;
    const uint64_t s = ok ? uint64_t(seg) : 0;
    const int d = __popcll((unsigned long long)s);
    int label = ok ? segment_label(s, c, m, k, ks) : -1;
    if (use_end && ok && c >= d && c < d + k) label = end.order[c - d];
    double col[MM];
    // rows d..d+k-1 and the squared sums below them are all the walk needs
    segment_qr<MM>(R0, stats->scale, m, label, c, col, piv_col[hw], min(m, d + k));

    if (!ok || c < d || c >= m) return;
    const int l = label < k ? label : c - d;  // column slot of this variable
    TO *an = anchor + seg * int64_t(k) * 32;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        const int r = i - d;
        if (r >= 0 && r < k) an[r * 32 + l] = TO(col[i]);
        if (r >= k) t = fma(col[i], col[i], t);
    }
    if (tail) tail[seg * 32 + l] = TO(t);
}

// Anchors of many datasets in one launch: half-wave h of the launch takes the
// segment h - seg_prefix[b] of dataset b, seg_prefix[b] <= h < seg_prefix[b+1].
template <int MM>
__global__ __launch_bounds__(256) void anchor_batched_kernel(const BatchItem *__restrict__ items,
                                                             const int64_t *__restrict__ seg_prefix,
                                                             int count, int64_t total_segs) {
    __shared__ double piv_col[ANCHOR_HALVES][MM];
    const int hw = threadIdx.x >> 5;
    const int c = threadIdx.x & 31;
    const int64_t gseg = int64_t(blockIdx.x) * ANCHOR_HALVES + hw;
    const bool ok = gseg < total_segs;
    int lo = 0, hi = count - 1;  // last b with seg_prefix[b] <= gseg
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_prefix[mid] <= gseg) lo = mid;
        else hi = mid - 1;
    }
    const BatchItem &d = items[lo];
    const int64_t seg = ok ? gseg - seg_prefix[lo] : 0;
    const uint64_t s = uint64_t(seg);
    const int dd = __popcll((unsigned long long)s);
    const int label = ok ? segment_label(s, c, d.m, d.k, d.ks) : -1;
    double col[MM];
    segment_qr<MM>(d.R0, d.stats->scale, ok ? d.m : 0, label, c, col, piv_col[hw],
                   ok ? min(d.m, dd + d.k) : 0);
    if (!ok || c < dd || c >= d.m) return;
    const int l = label < d.k ? label : c - dd;
    float *an = static_cast<float *>(const_cast<void *>(d.anchor)) + seg * int64_t(d.k) * 32;
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        const int r = i - dd;
        if (r >= 0 && r < d.k) an[r * 32 + l] = float(col[i]);
        if (r >= d.k) t = fma(col[i], col[i], t);
    }
    static_cast<float *>(const_cast<void *>(d.tail))[seg * 32 + l] = float(t);
}

hipError_t launch_anchors_batched_f32(const BatchItem *items, const int64_t *seg_prefix, int count,
                                      int64_t total_segs, int mmax, hipStream_t s) {
    const dim3 grid(unsigned((total_segs + ANCHOR_HALVES - 1) / ANCHOR_HALVES)), block(256);
    switch ((mmax + 3) / 4 * 4) {
#define GS_ABAT_CASE(MMV)                                                                      \
    case MMV:                                                                                  \
        hipLaunchKernelGGL((anchor_batched_kernel<MMV>), grid, block, 0, s, items, seg_prefix, \
                           count, total_segs);                                                 \
        break;
        GS_ABAT_CASE(4)
        GS_ABAT_CASE(8)
        GS_ABAT_CASE(12)
        GS_ABAT_CASE(16)
        GS_ABAT_CASE(20)
        GS_ABAT_CASE(24)
        GS_ABAT_CASE(28)
        GS_ABAT_CASE(32)
#undef GS_ABAT_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TO>
static hipError_t launch_anchors_impl(const double *R0, const ColStats *stats, int m, int k,
                                      int ks, int64_t nseg, TO *anchor, TO *tail,
                                      const WalkEnd &end, int use_end, hipStream_t s) {
    const dim3 grid(unsigned((nseg + ANCHOR_HALVES - 1) / ANCHOR_HALVES)), block(256);
    const int mm = (m + 3) / 4 * 4;
    switch (mm) {
#define GS_ANCHOR_CASE(MMV)                                                                   \
    case MMV:                                                                                 \
        hipLaunchKernelGGL((anchor_kernel<MMV, TO>), grid, block, 0, s, R0, stats, m, k, ks, \
                           nseg, anchor, tail, end, use_end);                                 \
        break;
        GS_ANCHOR_CASE(4)
        GS_ANCHOR_CASE(8)
        GS_ANCHOR_CASE(12)
        GS_ANCHOR_CASE(16)
        GS_ANCHOR_CASE(20)
        GS_ANCHOR_CASE(24)
        GS_ANCHOR_CASE(28)
        GS_ANCHOR_CASE(32)
#undef GS_ANCHOR_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TO>
hipError_t launch_anchors(const double *R0, const ColStats *stats, int m, int k, int ks,
                          int64_t nseg, TO *anchor, TO *tail, hipStream_t s) {
    return launch_anchors_impl<TO>(R0, stats, m, k, ks, nseg, anchor, tail, WalkEnd{}, 0, s);
}

template <typename TO>
hipError_t launch_anchors_end(const double *R0, const ColStats *stats, int m, int k, int ks,
                              int64_t nseg, const WalkEnd &end, TO *anchor, hipStream_t s) {
    return launch_anchors_impl<TO>(R0, stats, m, k, ks, nseg, anchor, nullptr, end, 1, s);
}

template hipError_t launch_anchors<float>(const double *, const ColStats *, int, int, int, int64_t,
                                          float *, float *, hipStream_t);
template hipError_t launch_anchors<double>(const double *, const ColStats *, int, int, int, int64_t,
                                           double *, double *, hipStream_t);
template hipError_t launch_anchors_end<float>(const double *, const ColStats *, int, int, int,
                                              int64_t, const WalkEnd &, float *, hipStream_t);
template hipError_t launch_anchors_end<double>(const double *, const ColStats *, int, int, int,
                                               int64_t, const WalkEnd &, double *, hipStream_t);

}  // namespace gs
