// Segment anchors: the R factor each segment's walk starts from (FP64).
//
// Sec. 6 gives every processor its own initial QRD but not how to form it.  A
// segment's ordering is [front variables, middle block, inner block, back
// variables]; since X P = Q0 (R0 P), the R of that ordering equals (up to row
// signs) the R of QR(R0 P), an m x m Householder QR instead of an n x m one.
// Rows of the front variables never change during the walk and are dropped;
// rows of the back variables never change either and only enter through their
// squared sums (the "tail" of each back column).
//
// Output layout, per segment s, in "lane" order (lane l < k holds the column of
// variable l, lane k + i the i-th back variable in ascending label order):
//   anchor[s][r][l], r = 0..k-1 local rows (first the q middle rows, then the ks
//                    inner rows), l = 0..31
//   tail[s][l]     = sum of squares of column l over the back rows.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs_internal.hpp"

namespace gs {

__global__ __launch_bounds__(64) void anchor_kernel(const double *__restrict__ R0, int m, int k,
                                                    int ks, int64_t nseg,
                                                    double *__restrict__ anchor,
                                                    double *__restrict__ tail) {
    __shared__ double A[32][33];
    __shared__ int pos_label[32];
    const int64_t seg = blockIdx.x;
    const int lane = threadIdx.x;
    const int q = k - ks, nout = m - k;
    if (seg >= nseg) return;
    const int d = __popcll((unsigned long long)seg);
    if (lane == 0) {
        int pos = 0;
        for (int b = nout - 1; b >= 0; --b)
            if ((seg >> b) & 1) pos_label[pos++] = k + b;  // front, descending labels
        for (int p = 0; p < q; ++p) pos_label[pos++] = ks + p;  // middle
        for (int i = 0; i < ks; ++i) pos_label[pos++] = i;      // inner
        for (int b = 0; b < nout; ++b)
            if (!((seg >> b) & 1)) pos_label[pos++] = k + b;  // back, ascending
    }
    __syncthreads();
    for (int e = lane; e < m * m; e += 64) {
        const int r = e / m, c = e - (e / m) * m;
        A[r][c] = R0[r * m + pos_label[c]];
    }
    __syncthreads();
    // Householder QR of R0 P, one column per lane.
    for (int j = 0; j < m; ++j) {
        const double a = A[j][j];
        double tailn = 0.0;
        for (int i = j + 1; i < m; ++i) tailn += A[i][j] * A[i][j];
        const double normx2 = tailn + a * a;
        double alpha = a;
        if (normx2 > 0.0) {
            const double nrm = sqrt(normx2);
            alpha = a >= 0.0 ? -nrm : nrm;
            const double v0 = a - alpha;
            const double vtv = tailn + v0 * v0;
            if (lane > j && lane < m) {
                double dot = v0 * A[j][lane];
                for (int i = j + 1; i < m; ++i) dot += A[i][j] * A[i][lane];
                const double f = 2.0 * dot / vtv;
                A[j][lane] -= f * v0;
                for (int i = j + 1; i < m; ++i) A[i][lane] -= f * A[i][j];
            }
        }
        __syncthreads();
        if (lane == j) {
            A[j][j] = alpha;
            for (int i = j + 1; i < m; ++i) A[i][j] = 0.0;
        }
        __syncthreads();
    }
    if (lane >= 32) return;
    int pos = -1;
    if (lane < ks) pos = d + q + lane;
    else if (lane < k) pos = d + (lane - ks);
    else if (lane < k + (nout - d)) pos = d + lane;  // back variables follow the k walked ones
    double *an = anchor + seg * int64_t(k) * 32;
    for (int r = 0; r < k; ++r) an[r * 32 + lane] = pos >= 0 ? A[d + r][pos] : 0.0;
    double t = 0.0;
    if (pos >= 0)
        for (int r = d + k; r < m; ++r) t += A[r][pos] * A[r][pos];
    tail[seg * 32 + lane] = t;
}

hipError_t launch_anchors(const double *R0, int m, int k, int ks, int64_t nseg, double *anchor,
                          double *tail, hipStream_t s) {
    hipLaunchKernelGGL(anchor_kernel, dim3(unsigned(nseg)), dim3(64), 0, s, R0, m, k, ks, nseg,
                       anchor, tail);
    return hipGetLastError();
}

}  // namespace gs
