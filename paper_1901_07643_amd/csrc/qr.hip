// R0 = triangular factor of the QR decomposition of the data X (FP64).
//
// The paper starts from one QRD of the n x m data (Sec. 2) and counts it as the
// O(2 n m^2) step of Sec. 1.1.  Here it is a tall-skinny QR: every workgroup
// triangularises a block of 128 rows by Householder reflections and writes its
// m x m R; the stacked R blocks are triangularised again by the same code until one
// block is left.  The first pass flags non-finite input and scales each column of its
// block by the power of two that brings the block's largest magnitude into [1/2, 1),
// so that no square or sum of squares of the QR leaves the double range whatever the
// units of X; it records those exponents and raises the column's global exponent
// exp0 to the largest of them.  The next pass brings every block's R to the common
// scale 2^-exp0 by exact powers of two (the same numbers as a pre-scaling of all of X
// by 2^-exp0 would give).  The last pass makes the diagonal non-negative, derives the
// column statistics the later stages use (the walk's power-of-two equilibration,
// variance inflation factors) and checks the rank.
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

#include <climits>
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

// Column statistics (lane c of the first 32 threads handles column c), from the
// signed R0 of the pre-scaled data X 2^-exp0 in Rl (zero outside the m x m upper
// triangle):
//   scale[c] = 2^-e: column c of that R0 times scale[c] has a norm in [1/2, 1), and
//     exp2[c] = exp0[c] + e: the column of X times 2^-exp2[c] has that norm;
//   vif[c] = ||x_c||^2 [(R0^T R0)^-1]_cc = ||x_c||^2 / RSS(c | all other columns),
//     from the rows of (R0 D)^-1 (D = diag(scale)); inf for a singular R0.
// Rank flag (scale-free): some column within an angle of n eps of the span of the
// columns before it (r_cc / ||x_c||) or of all others (1 / sqrt(vif)).  The walks take
// their guarded Givens steps when the rank flag is set or the largest vif exceeds
// GS_GUARD_VIF; below that every pivot pair of the equilibrated walk is far from
// zero and from the FP32 underflow threshold.
template <int MM>
__device__ __forceinline__ void col_stats(double (*Rl)[QR_MMAX + 1], const int *exps, int m,
                                          int64_t n, int *__restrict__ status,
                                          ColStats *__restrict__ st) {
    __shared__ double scl[QR_MMAX];
    __shared__ double Zl[QR_MMAX][QR_MMAX + 1];
    const int c = threadIdx.x;  // 0..31
    double sc = 1.0, ns = 0.0;
    if (c < m) {
        // the column's norm is at least its largest entry's magnitude, which the
        // pre-scaling put in [1/2, 1) (a zero column keeps scale 1 and norm 0)
        double t = 0.0;
        for (int i = 0; i <= c; ++i) t = fma(Rl[i][c], Rl[i][c], t);
        int e = 0;
        if (t > 0.0) {
            (void)frexp(sqrt(t), &e);
            sc = ldexp(1.0, -e);
            ns = ldexp(sqrt(t), -e);
        }
        const int e0 = exps[c];
        st->exp2[c] = (e0 == INT_MIN ? 0 : e0) + e;
        st->scale[c] = sc;
    }
    scl[c] = c < m ? sc : 0.0;
    wave_lds_sync();
    // column c of (R0 D)^-1 by back substitution (zero below row c)
    double z[MM];
#pragma unroll
    for (int i = MM - 1; i >= 0; --i) {
        double v = 0.0;
        if (i <= c && c < m) {
            double acc = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int l = i + 1; l < MM; ++l) acc = fma(-Rl[i][l] * scl[l], z[l], acc);
            v = acc / (Rl[i][i] * scl[i]);
        }
        z[i] = v;
    }
#pragma unroll
    for (int i = 0; i < MM; ++i) Zl[c][i] = z[i];
    wave_lds_sync();
    double vif = 0.0, dang = 1.0;
    if (c < m) {
        double w = 0.0;
        for (int j = c; j < m; ++j) w = fma(Zl[j][c], Zl[j][c], w);
        vif = ns * ns * w;
        if (!(vif < INFINITY)) vif = INFINITY;  // singular: inf or NaN from 0 / 0
        st->vif[c] = vif;
        dang = ns > 0.0 ? fabs(Rl[c][c] * sc) / ns : 0.0;
    }
    double vmax = vif, dmin = dang;
#pragma unroll
    for (int off = 16; off >= 1; off >>= 1) {
        vmax = fmax(vmax, __shfl_xor(vmax, off, 32));
        dmin = fmin(dmin, __shfl_xor(dmin, off, 32));
    }
    if (c == 0) {
        const double tau = double(n) * 2.220446049250313e-16;
        int f = 0;
        if (!(dmin > tau) || !(vmax * tau * tau < 1.0)) f = GS_FLAG_RANK | GS_FLAG_GUARD;
        else if (!(vmax < GS_GUARD_VIF)) f = GS_FLAG_GUARD;
        if (f) atomicOr(status, f);
    }
}

__global__ void front_reset_kernel(int *__restrict__ status, ColStats *__restrict__ stats,
                                   int count) {
    for (int i = int(blockIdx.x * blockDim.x + threadIdx.x); i < count * 32;
         i += int(gridDim.x * blockDim.x)) {
        if ((i & 31) == 0) status[i >> 5] = 0;
        stats[i >> 5].exp0[i & 31] = INT_MIN;
    }
}

// One 128-row block: A (nrows x m, row stride lda) rows [r0, r0 + 128) -> Rout (m x m).
// The first pass (first != 0) reads X: it checks every entry, scales column c of the
// block by 2^-e (e: the exponent of the block's largest |x_ic|, or INT_MIN for an
// all-zero column), stores e at eblk[block][c] and raises stats->exp0[c] to it.  The
// pass after it (rescale != 0) reads those blocks' R factors, row i of A belonging to
// block i / m, and multiplies each column by 2^(e - exp0).
template <int MM>
__device__ __forceinline__ void tsqr_block(const double *__restrict__ A, int64_t nrows, int m,
                                           int64_t lda, int64_t r0, int block,
                                           double *__restrict__ Rout, double *__restrict__ Rtrue,
                                           int *__restrict__ status, ColStats *__restrict__ stats,
                                           int first, int rescale, int *__restrict__ eblk,
                                           int final_pass, int64_t n_orig) {
    // per column parity: partial dot products of the 8 row groups, row j, pivot entry
    __shared__ double red[2][QR_G][QR_MMAX];
    __shared__ double rowj[2][QR_MMAX];
    __shared__ double diag[QR_MMAX];
    __shared__ int exps[QR_MMAX];  // the exponents of the common scale (final pass)
    const int tid = threadIdx.x;
    const int c = tid & 31;   // column
    const int g = tid >> 5;   // row group
    const int rows = int(min<int64_t>(QR_BR, nrows - r0));

    double x[QR_RPT];
#pragma unroll
    for (int r = 0; r < QR_RPT; ++r) {
        const int i = g + QR_G * r;
        x[r] = (i < rows && c < m) ? A[(r0 + i) * lda + c] : 0.0;
    }
    if (first) {
        double mx = 0.0;
        int bad = 0;
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) {
            if (!isfinite(x[r])) bad = 1;
            mx = fmax(mx, fabs(x[r]));  // fmax ignores a NaN operand
        }
        if (bad) atomicOr(status, GS_FLAG_NOTFINITE);
        red[0][g][c] = mx;
        __syncthreads();
#pragma unroll
        for (int gg = 0; gg < QR_G; ++gg) mx = fmax(mx, red[0][gg][c]);
        int e = INT_MIN;
        if (mx > 0.0 && mx <= 1.7976931348623157e308) (void)frexp(mx, &e);
        if (g == 0 && c < m) {
            if (e != INT_MIN) atomicMax(stats->exp0 + c, e);
            if (final_pass) exps[c] = e;
            else eblk[block * 32 + c] = e;
        }
        const int sh = e == INT_MIN ? 0 : -e;
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) x[r] = ldexp(x[r], sh);
        __syncthreads();  // the maxima are read before the QR reuses red
    } else if (rescale && c < m) {
        const int E = stats->exp0[c];
#pragma unroll
        for (int r = 0; r < QR_RPT; ++r) {
            const int i = g + QR_G * r;
            if (i < rows) {
                const int e = eblk[int((r0 + i) / m) * 32 + c];
                x[r] = e == INT_MIN ? 0.0 : ldexp(x[r], e - E);
            }
        }
    }
    if (final_pass && !first && g == 0 && c < m) exps[c] = stats->exp0[c];

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
    // the signed R0, zero outside the m x m triangle, for the statistics below
    __shared__ double Rl[QR_MMAX][QR_MMAX + 1];
    for (int e = tid; e < QR_MMAX * (QR_MMAX + 1); e += QR_THREADS) (&Rl[0][0])[e] = 0.0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QR_RPT; ++r) {
        const int i = g + QR_G * r;
        if (i < m && c < m) {
            double val = (i < rows && c >= i) ? x[r] : 0.0;
            if (diag[i] < 0.0) val = -val;
            Rout[i * m + c] = val;
            Rl[i][c] = val;
            if (Rtrue) {
                const int e = exps[c];
                Rtrue[i * m + c] = ldexp(val, e == INT_MIN ? 0 : e);
            }
        }
    }
    __syncthreads();
    if (tid < 32) col_stats<MM>(Rl, exps, m, n_orig, status, stats);
}

template <int MM>
__global__ __launch_bounds__(QR_THREADS) void tsqr_block_kernel(
    const double *__restrict__ A, int64_t nrows, int m, int64_t lda, double *__restrict__ Rout,
    double *__restrict__ Rtrue, int *__restrict__ status, ColStats *__restrict__ stats, int first,
    int rescale, int *__restrict__ eblk, int final_pass, int64_t n_orig) {
    tsqr_block<MM>(A, nrows, m, lda, int64_t(blockIdx.x) * QR_BR, int(blockIdx.x),
                   Rout + int64_t(blockIdx.x) * m * m, Rtrue, status, stats, first, rescale, eblk,
                   final_pass, n_orig);
}

// Batched passes: one job per workgroup (see TsqrJob); MM covers the largest m.
template <int MM>
__global__ __launch_bounds__(QR_THREADS) void tsqr_batched_kernel(const TsqrJob *__restrict__ jobs,
                                                                  int njobs) {
    if (int(blockIdx.x) >= njobs) return;
    const TsqrJob jb = jobs[blockIdx.x];
    tsqr_block<MM>(jb.A, jb.nrows, jb.m, jb.lda, int64_t(jb.block) * QR_BR, jb.block, jb.Rout,
                   nullptr, jb.status, jb.stats, jb.first, jb.rescale, jb.eblk, jb.final_pass,
                   jb.n_orig);
}

// Per buffer: the R blocks of the first pass, then (first buffer only) their column
// exponents, 32 ints per block.
int64_t qr_workspace_elems(int64_t n, int m) {
    const int64_t nb = (n + QR_BR - 1) / QR_BR;
    return nb * int64_t(m) * m + int64_t(m) * m + 16 * nb;
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
                               double *Rtrue, int *status, ColStats *stats, int first,
                               int rescale, int *eblk, int final_pass, int64_t n, int64_t nb,
                               hipStream_t s) {
#define GS_QR_CASE(MMV)                                                                        \
    case MMV:                                                                                  \
        hipLaunchKernelGGL((tsqr_block_kernel<MMV>), dim3(unsigned(nb)), dim3(QR_THREADS), 0, s, \
                           A, rows, m, lda, Rout, Rtrue, status, stats, first, rescale, eblk,  \
                           final_pass, n);                                                     \
        break;
    GS_QR_SWITCH((m + 3) / 4 * 4, GS_QR_CASE)
#undef GS_QR_CASE
    return hipGetLastError();
}

hipError_t launch_front_reset(int *status, ColStats *stats, int count, hipStream_t s) {
    const int threads = 256, blocks = (count * 32 + threads - 1) / threads;
    hipLaunchKernelGGL(front_reset_kernel, dim3(unsigned(blocks)), dim3(threads), 0, s, status,
                       stats, count);
    return hipGetLastError();
}

hipError_t launch_qr_r0(const double *X, int64_t n, int m, int64_t ldx, double *R0, double *Rtrue,
                        double *bufA, double *bufB, int *status, ColStats *stats, hipStream_t s) {
    const int64_t nb0 = (n + QR_BR - 1) / QR_BR;
    // the first pass's block exponents, behind the largest R stack in bufA
    int *eblk = reinterpret_cast<int *>(bufA + nb0 * int64_t(m) * m + int64_t(m) * m);
    const double *src = X;
    int64_t rows = n, lda = ldx;
    double *dst = bufA, *other = bufB;
    int first = 1, rescale = 0;
    for (;;) {
        const int64_t nb = (rows + QR_BR - 1) / QR_BR;
        if (nb == 1)
            return launch_block(src, rows, m, lda, R0, Rtrue, status, stats, first, rescale, eblk,
                                1, n, 1, s);
        hipError_t e = launch_block(src, rows, m, lda, dst, nullptr, status, stats, first, rescale,
                                    eblk, 0, n, nb, s);
        if (e != hipSuccess) return e;
        rescale = first;
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
