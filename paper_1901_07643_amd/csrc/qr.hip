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
// (g, c) keeps column c of the rows i = g + 8 r, r = 0..15, in registers.  The
// column loop is unrolled with the column index j known at compile time (the kernel
// is instantiated for MM = m rounded up to a multiple of 4), so that the rows above
// the pivot are skipped without run-time tests.  A Householder step broadcasts the
// pivot column inside each row group with ds_bpermute, forms the partial dot
// products and combines the 8 groups through LDS; the LDS buffers alternate
// between even and odd columns, so one workgroup barrier per column suffices.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gs_internal.hpp"

namespace gs {

constexpr int QR_BR = 128;      // rows per workgroup
constexpr int QR_THREADS = 256;
constexpr int QR_G = 8;         // row groups
constexpr int QR_RPT = QR_BR / QR_G;  // rows per thread
constexpr int QR_MMAX = 32;     // columns (m <= 30)

template <int I, int N, typename Fn>
__device__ __forceinline__ void qr_static_for(Fn &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        qr_static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ double shfl_half(double v, int src) {
    return __shfl(v, src, 32);
}

// One 128-row block: A (nrows x m, row stride lda) rows [r0, r0 + 128) -> Rout (m x m).
template <int MM>
__device__ __forceinline__ void tsqr_block(const double *__restrict__ A, int64_t nrows, int m,
                                           int64_t lda, int64_t r0, double *__restrict__ Rout,
                                           int *__restrict__ status, int check_finite,
                                           int final_pass, int64_t n_orig) {
    // per column parity: partial dot products of the 8 row groups, row j, pivot entry
    __shared__ double red[2][QR_G][QR_MMAX];
    __shared__ double rowj[2][QR_MMAX];
    __shared__ double diag[QR_MMAX];
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

    // Rows past the block's end hold zeros; a column j >= rows then has a zero
    // tail and its step leaves every row unchanged (normx2 = a^2 with a = 0 below the
    // block, or the step is a plain sign normalisation).
    qr_static_for<0, MM>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        constexpr int gj = j % QR_G, rj = j / QR_G;  // owner of row j
        constexpr int par = j & 1;
        if (j < m) {
            double v[QR_RPT];
            double part = 0.0;
#pragma unroll
            for (int r = rj; r < QR_RPT; ++r) {
                v[r] = shfl_half(x[r], j);
                if (r > rj || g > gj) part = fma(v[r], x[r], part);
            }
            red[par][g][c] = part;
            if (g == gj) rowj[par][c] = x[rj];
            __syncthreads();
            double P = 0.0, tailn = 0.0;
#pragma unroll
            for (int gg = 0; gg < QR_G; ++gg) {
                P += red[par][gg][c];
                tailn += red[par][gg][j];
            }
            const double a = rowj[par][j];
            const double rj_c = rowj[par][c];
            const double normx2 = fma(a, a, tailn);
            if (normx2 > 0.0) {
                // normx2 is the same in every thread, so the branch is uniform
                double nrm, rvtv;
                // (bounded above too, so that 1 / v^T v <= 1 / normx2 stays a normal number)
                const bool normal = normx2 >= GS_DBL_MIN && normx2 <= 1e300;
                if (normal) nrm = normx2 * rsq_newton(normx2);
                else nrm = sqrt(normx2);
                const double alpha = a >= 0.0 ? -nrm : nrm;
                const double v0 = a - alpha;
                const double vtv = fma(v0, v0, tailn);
                if (normal) rvtv = rcp_newton(vtv);
                else rvtv = 1.0 / vtv;
                const double f = (c > j && c < m) ? 2.0 * fma(v0, rj_c, P) * rvtv : 0.0;
#pragma unroll
                for (int r = rj + 1; r < QR_RPT; ++r) x[r] = fma(-f, v[r], x[r]);
                if (g > gj) x[rj] = fma(-f, v[rj], x[rj]);
                else if (g == gj) x[rj] = (c == j) ? alpha : fma(-f, v0, x[rj]);
            }
        }
    });

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

template <int MM>
__global__ __launch_bounds__(QR_THREADS) void tsqr_block_kernel(const double *__restrict__ A,
                                                                int64_t nrows, int m, int64_t lda,
                                                                double *__restrict__ Rout,
                                                                int *__restrict__ status,
                                                                int check_finite, int final_pass,
                                                                int64_t n_orig) {
    tsqr_block<MM>(A, nrows, m, lda, int64_t(blockIdx.x) * QR_BR,
                   Rout + int64_t(blockIdx.x) * m * m, status, check_finite, final_pass, n_orig);
}

// Batched passes: one job per workgroup (see TsqrJob); MM covers the largest m.
template <int MM>
__global__ __launch_bounds__(QR_THREADS) void tsqr_batched_kernel(const TsqrJob *__restrict__ jobs,
                                                                  int njobs) {
    if (int(blockIdx.x) >= njobs) return;
    const TsqrJob jb = jobs[blockIdx.x];
    tsqr_block<MM>(jb.A, jb.nrows, jb.m, jb.lda, int64_t(jb.block) * QR_BR, jb.Rout, jb.status,
                   jb.check_finite, jb.final_pass, jb.n_orig);
}

int64_t qr_workspace_elems(int64_t n, int m) {
    const int64_t nb = (n + QR_BR - 1) / QR_BR;
    return nb * int64_t(m) * m + int64_t(m) * m;
}

int tsqr_rows_per_block() { return QR_BR; }

#define GS_QR_SWITCH(MMV_EXPR, CASE) \
    switch (MMV_EXPR) {                \
        CASE(4)                        \
        CASE(8)                        \
        CASE(12)                       \
        CASE(16)                       \
        CASE(20)                       \
        CASE(24)                       \
        CASE(28)                       \
        CASE(32)                       \
        default: return hipErrorInvalidValue; \
    }

static hipError_t launch_block(const double *A, int64_t rows, int m, int64_t lda, double *Rout,
                               int *status, int first, int final_pass, int64_t n, int64_t nb,
                               hipStream_t s) {
#define GS_QR_CASE(MMV)                                                                        \
    case MMV:                                                                                  \
        hipLaunchKernelGGL((tsqr_block_kernel<MMV>), dim3(unsigned(nb)), dim3(QR_THREADS), 0, s, \
                           A, rows, m, lda, Rout, status, first, final_pass, n);               \
        break;
    GS_QR_SWITCH((m + 3) / 4 * 4, GS_QR_CASE)
#undef GS_QR_CASE
    return hipGetLastError();
}

hipError_t launch_qr_r0(const double *X, int64_t n, int m, int64_t ldx, double *R0, double *bufA,
                        double *bufB, int *status, hipStream_t s) {
    const double *src = X;
    int64_t rows = n, lda = ldx;
    double *dst = bufA, *other = bufB;
    int first = 1;
    for (;;) {
        const int64_t nb = (rows + QR_BR - 1) / QR_BR;
        if (nb == 1) return launch_block(src, rows, m, lda, R0, status, first, 1, n, 1, s);
        hipError_t e = launch_block(src, rows, m, lda, dst, status, first, 0, n, nb, s);
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

hipError_t launch_tsqr_batched(const TsqrJob *jobs, int njobs, int mmax, hipStream_t s) {
#define GS_QRB_CASE(MMV)                                                                      \
    case MMV:                                                                                 \
        hipLaunchKernelGGL((tsqr_batched_kernel<MMV>), dim3(unsigned(njobs)), dim3(QR_THREADS), \
                           0, s, jobs, njobs);                                                \
        break;
    GS_QR_SWITCH((mmax + 3) / 4 * 4, GS_QRB_CASE)
#undef GS_QRB_CASE
    return hipGetLastError();
}
#undef GS_QR_SWITCH

}  // namespace gs
