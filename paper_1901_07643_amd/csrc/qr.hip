// R0 = triangular factor of the QR decomposition of the data X (FP64).
//
// The paper starts from one QRD of the n x m data (Sec. 2) and counts it as the
// O(2 n m^2) step of Sec. 1.1.  Here it is a tall-skinny QR: every workgroup
// triangularises a block of 128 rows by Householder reflections in LDS and writes
// its m x m R; the stacked R blocks are triangularised again by the same kernel
// until one block is left.  The last pass makes the diagonal non-negative and
// checks the rank.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs_internal.hpp"

namespace gs {

constexpr int QR_BR = 128;      // rows per workgroup
constexpr int QR_THREADS = 256;
constexpr int QR_MMAX = 32;     // columns held per row in LDS (m <= 30)

__global__ __launch_bounds__(QR_THREADS) void tsqr_block_kernel(const double *__restrict__ A,
                                                                int64_t nrows, int m, int64_t lda,
                                                                double *__restrict__ Rout,
                                                                int *__restrict__ status,
                                                                int check_finite, int final_pass,
                                                                int64_t n_orig) {
    __shared__ double S[QR_BR][QR_MMAX + 1];
    __shared__ double red[QR_THREADS / 32][QR_MMAX];
    __shared__ double P[QR_MMAX];
    __shared__ double F[QR_MMAX];
    __shared__ double sc[2];  // alpha, skip flag
    const int tid = threadIdx.x;
    const int64_t r0 = int64_t(blockIdx.x) * QR_BR;
    const int rows = int(min<int64_t>(QR_BR, nrows - r0));

    int bad = 0;
    for (int e = tid; e < QR_BR * m; e += QR_THREADS) {
        const int i = e / m, c = e - (e / m) * m;
        double v = 0.0;
        if (i < rows) {
            v = A[(r0 + i) * lda + c];
            if (check_finite && !isfinite(v)) bad = 1;
        }
        S[i][c] = v;
    }
    if (bad) atomicOr(status, GS_FLAG_NOTFINITE);
    __syncthreads();

    const int ct = tid & 31;  // column handled in the 2-D loops
    const int g = tid >> 5;   // row group 0..7
    constexpr int G = QR_THREADS / 32;
    const int steps = min(m, rows);
    for (int j = 0; j < steps; ++j) {
        // P[c] = sum_{i > j} S[i][j] S[i][c] for c >= j
        double part = 0.0;
        if (ct >= j && ct < m)
            for (int i = j + 1 + g; i < rows; i += G) part += S[i][j] * S[i][ct];
        red[g][ct] = part;
        __syncthreads();
        if (tid < QR_MMAX) {
            double s = 0.0;
            for (int gg = 0; gg < G; ++gg) s += red[gg][tid];
            P[tid] = s;
        }
        __syncthreads();
        if (tid < QR_MMAX) {
            const double a = S[j][j];
            const double tailn = P[j];
            const double normx2 = tailn + a * a;
            double f = 0.0, alpha = a, skip = 1.0;
            if (normx2 > 0.0) {
                const double nrm = sqrt(normx2);
                alpha = a >= 0.0 ? -nrm : nrm;
                const double v0 = a - alpha;
                const double vtv = tailn + v0 * v0;
                skip = 0.0;
                if (tid > j && tid < m) f = 2.0 * (v0 * S[j][tid] + P[tid]) / vtv;
                if (tid == 0) sc[0] = alpha;
                // v0 is needed by the row-j update: keep it in F[j]
                if (tid == j) F[j] = v0;
            }
            if (tid != j) F[tid] = f;
            if (tid == 0) sc[1] = skip;
        }
        __syncthreads();
        if (sc[1] == 0.0) {
            if (ct > j && ct < m) {
                const double f = F[ct];
                for (int i = j + 1 + g; i < rows; i += G) S[i][ct] -= f * S[i][j];
                if (g == 0) S[j][ct] -= f * F[j];
            }
            __syncthreads();
            if (tid == 0) S[j][j] = sc[0];
        }
        __syncthreads();
    }

    double *R = Rout + int64_t(blockIdx.x) * m * m;
    if (!final_pass) {
        for (int e = tid; e < m * m; e += QR_THREADS) {
            const int r = e / m, c = e - (e / m) * m;
            R[e] = (r < rows && c >= r) ? S[r][c] : 0.0;
        }
        return;
    }
    // final block: non-negative diagonal, rank check
    for (int e = tid; e < m * m; e += QR_THREADS) {
        const int r = e / m, c = e - (e / m) * m;
        double v = 0.0;
        if (r < rows && c >= r) {
            v = S[r][c];
            if (S[r][r] < 0.0) v = -v;
        }
        R[e] = v;
    }
    if (tid == 0) {
        double dmax = 0.0, dmin = INFINITY;
        for (int r = 0; r < m; ++r) {
            const double d = r < rows ? fabs(S[r][r]) : 0.0;
            dmax = fmax(dmax, d);
            dmin = fmin(dmin, d);
        }
        const double eps = 2.220446049250313e-16;
        if (!(dmin > double(n_orig) * eps * dmax)) atomicOr(status, GS_FLAG_RANK);
    }
}

int64_t qr_workspace_elems(int64_t n, int m) {
    const int64_t nb = (n + QR_BR - 1) / QR_BR;
    return nb * int64_t(m) * m + int64_t(m) * m;
}

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

}  // namespace gs
