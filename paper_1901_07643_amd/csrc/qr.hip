// R0 = triangular factor of the QR decomposition of the data X (FP64).
//
// The paper starts from one QRD of the n x m data (Sec. 2) and counts it as the
// O(2 n m^2) step of Sec. 1.1.  Here it is a tall-skinny QR: every workgroup
// triangularises a block of 128 rows by Householder reflections and writes its
// m x m R; the stacked R blocks are triangularised again by the same code until one
// block is left.  The last pass makes the diagonal non-negative and checks the rank;
// the first pass flags non-finite input.
//
// Layout inside a workgroup (256 threads = 8 row groups x 32 columns): thread
// (g, c) keeps column c of the rows i = g + 8 r, r = 0..15, in registers.  A
// Householder step broadcasts the pivot column inside each row group with
// ds_bpermute, forms the partial dot products, and combines the 8 groups through LDS:
// two workgroup barriers per column.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs_internal.hpp"

namespace gs {

constexpr int QR_BR = 128;      // rows per workgroup
constexpr int QR_THREADS = 256;
constexpr int QR_G = 8;         // row groups
constexpr int QR_RPT = QR_BR / QR_G;  // rows per thread
constexpr int QR_MMAX = 32;     // columns (m <= 30)

__device__ __forceinline__ double shfl_half(double v, int src) {
    return __shfl(v, src, 32);
}

// One 128-row block: A (nrows x m, row stride lda) rows [r0, r0 + 128) -> Rout (m x m).
__device__ __forceinline__ void tsqr_block(const double *__restrict__ A, int64_t nrows, int m,
                                           int64_t lda, int64_t r0, double *__restrict__ Rout,
                                           int *__restrict__ status, int check_finite,
                                           int final_pass, int64_t n_orig) {
    __shared__ double red[QR_G][QR_MMAX];
    __shared__ double rowj[QR_MMAX];
    __shared__ double diag[QR_MMAX];
    __shared__ double piv_a;
    const int tid = threadIdx.x;
    const int c = tid & 31;   // column
    const int g = tid >> 5;   // row group
    const int rows = int(min<int64_t>(QR_BR, nrows - r0));

    double x[QR_RPT];
    int bad = 0;
#pragma unroll
    for (int r = 0; r < QR_RPT; ++r) {
        const int i = g + QR_G * r;
        double v = 0.0;
        if (i < rows && c < m) {
            v = A[(r0 + i) * lda + c];
            if (check_finite && !isfinite(v)) bad = 1;
        }
        x[r] = v;
    }
    if (bad) atomicOr(status, GS_FLAG_NOTFINITE);

    const int steps = min(m, rows);
    for (int j = 0; j < steps; ++j) {
        const int gj = j % QR_G, rj = j / QR_G;  // owner of row j
        // pivot column entries of this thread's rows (from lane j of the row group)
        double v[QR_RPT];
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) v[r] = shfl_half(x[r], j);
        double part = 0.0;
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) {
            const int i = g + QR_G * r;
            if (i > j) part = fma(v[r], x[r], part);
        }
        red[g][c] = part;
        if (g == gj) {
#pragma unroll
            for (int r = 0; r < QR_RPT; ++r)
                if (r == rj) rowj[c] = x[r];
            if (c == j) piv_a = rowj[c];
        }
        __syncthreads();
        double P = 0.0, tailn = 0.0;
#pragma unroll
        for (int gg = 0; gg < QR_G; ++gg) {
            P += red[gg][c];
            tailn += red[gg][j];
        }
        const double a = piv_a;
        const double rj_c = rowj[c];
        __syncthreads();  // red / rowj / piv_a may be rewritten from here on
        const double normx2 = fma(a, a, tailn);
        if (normx2 > 0.0) {
            const double nrm = sqrt(normx2);
            const double alpha = a >= 0.0 ? -nrm : nrm;
            const double v0 = a - alpha;
            const double vtv = fma(v0, v0, tailn);
            const double f = (c > j && c < m) ? 2.0 * fma(v0, rj_c, P) / vtv : 0.0;
#pragma unroll
            for (int r = 0; r < QR_RPT; ++r) {
                const int i = g + QR_G * r;
                if (i > j) x[r] = fma(-f, v[r], x[r]);
                else if (i == j) x[r] = (c == j) ? alpha : fma(-f, v0, x[r]);
            }
        }
    }

    // rows 0..m-1 of the block's R (zero below the diagonal and past the block's rows)
    if (!final_pass) {
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) {
            const int i = g + QR_G * r;
            if (i < m && c < m) Rout[i * m + c] = (i < rows && c >= i) ? x[r] : 0.0;
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < QR_RPT; ++r) {
        const int i = g + QR_G * r;
        if (i < m && c == i) diag[i] = i < rows ? x[r] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QR_RPT; ++r) {
        const int i = g + QR_G * r;
        if (i < m && c < m) {
            double val = (i < rows && c >= i) ? x[r] : 0.0;
            if (diag[i] < 0.0) val = -val;
            Rout[i * m + c] = val;
        }
    }
    if (tid == 0) {
        double dmax = 0.0, dmin = INFINITY;
        for (int r = 0; r < m; ++r) {
            const double d = fabs(diag[r]);
            dmax = fmax(dmax, d);
            dmin = fmin(dmin, d);
        }
        const double eps = 2.220446049250313e-16;
        if (!(dmin > double(n_orig) * eps * dmax)) atomicOr(status, GS_FLAG_RANK);
    }
}

__global__ __launch_bounds__(QR_THREADS) void tsqr_block_kernel(const double *__restrict__ A,
                                                                int64_t nrows, int m, int64_t lda,
                                                                double *__restrict__ Rout,
                                                                int *__restrict__ status,
                                                                int check_finite, int final_pass,
                                                                int64_t n_orig) {
    tsqr_block(A, nrows, m, lda, int64_t(blockIdx.x) * QR_BR, Rout + int64_t(blockIdx.x) * m * m,
               status, check_finite, final_pass, n_orig);
}

// Batched passes: one job per workgroup (see TsqrJob).
__global__ __launch_bounds__(QR_THREADS) void tsqr_batched_kernel(const TsqrJob *__restrict__ jobs,
                                                                  int njobs) {
    if (int(blockIdx.x) >= njobs) return;
    const TsqrJob jb = jobs[blockIdx.x];
    tsqr_block(jb.A, jb.nrows, jb.m, jb.lda, int64_t(jb.block) * QR_BR, jb.Rout, jb.status,
               jb.check_finite, jb.final_pass, jb.n_orig);
}

int64_t qr_workspace_elems(int64_t n, int m) {
    const int64_t nb = (n + QR_BR - 1) / QR_BR;
    return nb * int64_t(m) * m + int64_t(m) * m;
}

int tsqr_rows_per_block() { return QR_BR; }

hipError_t launch_qr_r0(const double *X, int64_t n, int m, int64_t ldx, double *R0, double *bufA,
                        double *bufB, int *status, hipStream_t s) {
    const double *src = X;
    int64_t rows = n, lda = ldx;
    double *dst = bufA, *other = bufB;
    int first = 1;
    for (;;) {
        const int64_t nb = (rows + QR_BR - 1) / QR_BR;
        if (nb == 1) {
            hipLaunchKernelGGL(tsqr_block_kernel, dim3(1), dim3(QR_THREADS), 0, s, src, rows, m, lda,
                               R0, status, first, 1, n);
            return hipGetLastError();
        }
        hipLaunchKernelGGL(tsqr_block_kernel, dim3(unsigned(nb)), dim3(QR_THREADS), 0, s, src, rows,
                           m, lda, dst, status, first, 0, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        first = 0;
        src = dst;
        rows = nb * m;
        lda = m;
        double *t = dst;
        dst = other;
        other = t;
    }
}

hipError_t launch_tsqr_batched(const TsqrJob *jobs, int njobs, hipStream_t s) {
    hipLaunchKernelGGL(tsqr_batched_kernel, dim3(unsigned(njobs)), dim3(QR_THREADS), 0, s, jobs,
                       njobs);
    return hipGetLastError();
}

}  // namespace gs
