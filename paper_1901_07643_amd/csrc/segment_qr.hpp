// Device helpers shared by the anchor kernel and its adjoint: the R factor of a
// segment's starting ordering, and the reverse-mode rule of a QR decomposition.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gs_internal.hpp"

namespace gs {

template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for_q(Fn &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_q<I + 1, N>(f);
    }
}

// Variable at position c of segment s's ordering
//   [front variables (descending labels), middle ks..k-1, inner 0..ks-1, back (ascending)],
// where bit b of s puts variable k + b in front.  -1 for c >= m.
__device__ __forceinline__ int segment_label(uint64_t s, int c, int m, int k, int ks) {
    const int q = k - ks, nout = m - k;
    const int d = __popcll((unsigned long long)s);
    if (c >= m) return -1;
    if (c < d) {
        int cnt = 0, label = -1;
        for (int b = nout - 1; b >= 0; --b)
            if ((s >> b) & 1) {
                if (cnt == c) label = k + b;
                ++cnt;
            }
        return label;
    }
    if (c < d + q) return ks + (c - d);
    if (c < d + k) return c - d - q;
    int cnt = 0, label = -1;
    for (int b = 0; b < nout; ++b)
        if (!((s >> b) & 1)) {
            if (cnt == c - d - k) label = k + b;
            ++cnt;
        }
    return label;
}

// Householder QR of A = R0 D P (R0: m x m row-major, D = diag(colscale), the
// power-of-two column equilibration, P: the ordering of segment s), one column per
// lane of a 32-lane half-wave: on return col[i] = R[i][c] for the lane's column c,
// with a non-negative diagonal.  Lanes c >= m hold unit columns (R is padded with the
// identity up to MM).  pc: MM doubles of LDS for this half-wave.
// With steps < m only the first `steps` reflections are applied: rows 0..steps-1 are
// then final, and rows steps.. hold, per column, the same sum of squares as the
// triangular R (the remaining reflections act on those rows alone and keep it).
template <int MM>
__device__ __forceinline__ void segment_qr(const double *__restrict__ R0,
                                           const double *__restrict__ colscale, int m, int label,
                                           int c, double (&col)[MM], double *pc, int steps) {
    const double sc = label >= 0 ? colscale[label] : 1.0;
#pragma unroll
    for (int i = 0; i < MM; ++i)
        col[i] = label >= 0 ? (i < m ? R0[i * m + label] * sc : 0.0) : (i == c ? 1.0 : 0.0);
    static_for_q<0, MM>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j < steps) {
            wave_lds_sync();  // every lane has read the previous pivot column
            if (c == j) {
#pragma unroll
                for (int i = j; i < MM; ++i) pc[i] = col[i];
            }
            wave_lds_sync();  // lane j's column is visible to the whole wave
            double v[MM];
#pragma unroll
            for (int i = j; i < MM; ++i) v[i] = pc[i];
            // every lane's product with the pivot column below row j; on the pivot
            // lane it is the pivot column's squared norm below j, which the other
            // lanes take from there
            double dotp = 0.0;
#pragma unroll
            for (int i = j + 1; i < MM; ++i) dotp = fma(v[i], col[i], dotp);
            const double tailn = __shfl(dotp, j, 32);
            const double a = v[j];
            const double normx2 = fma(a, a, tailn);
            double alpha = a, f = 0.0, v0 = 0.0;
            if (normx2 > 0.0) {
                // normx2 is the same in every lane of the half-wave (uniform branch)
                double nrm, rvtv;
                // (bounded above too, so that 1 / v^T v <= 1 / normx2 stays a normal number)
                const bool normal = normx2 >= GS_DBL_MIN && normx2 <= 1e300;
                if (normal) nrm = normx2 * rsq_newton(normx2);
                else nrm = sqrt(normx2);
                alpha = a >= 0.0 ? -nrm : nrm;
                v0 = a - alpha;
                const double vtv = fma(v0, v0, tailn);
                if (normal) rvtv = rcp_newton(vtv);
                else rvtv = 1.0 / vtv;
                f = 2.0 * fma(v0, col[j], dotp) * rvtv;
            }
            if (c == j) {
                col[j] = alpha;
#pragma unroll
                for (int i = j + 1; i < MM; ++i) col[i] = 0.0;
            } else {
                col[j] = fma(-f, v0, col[j]);
#pragma unroll
                for (int i = j + 1; i < MM; ++i) col[i] = fma(-f, v[i], col[i]);
            }
        }
    });
    // row signs: make every diagonal entry non-negative
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < MM; ++i)
        if (c == i) pc[i] = col[i] < 0.0 ? -1.0 : 1.0;
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < MM; ++i) col[i] *= pc[i];
    wave_lds_sync();
}

// Reverse-mode rule of A = Q R (square, R upper triangular, Q orthogonal) with a
// cotangent Rbar on R and none on Q:  Abar = Q copyltu(R Rbar^T) R^-T, where
// copyltu(M) = tril(M) + tril(M, -1)^T.  Since Q = A R^-1 this is
//     Abar = A V,   V = R^-1 copyltu(R Rbar^T) R^-T   (symmetric).
// The caller stores column c of R and of Rbar (zero below the diagonal) from lane c:
// qr_adj_store; qr_adjoint_core then leaves vrow[p] = V[c][p] (row c of V) in lane c.
// lds: 3 x MM x (MM+1) doubles belonging to this half-wave.
template <int MM>
__device__ __forceinline__ void qr_adj_store(const double (&col)[MM], const double (&rbar)[MM],
                                             int c, double *lds) {
    constexpr int LD = MM + 1;
    wave_lds_sync();
    if (c < MM) {
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            lds[i * LD + c] = col[i];
            lds[MM * LD + i * LD + c] = rbar[i];
        }
    }
    wave_lds_sync();
}

template <int MM>
__device__ __forceinline__ void qr_adjoint_core(int c, double *lds, double (&vrow)[MM]) {
    constexpr int LD = MM + 1;
    const double *Rl = lds;  // R[i][j] at Rl[i * LD + j]
    double *Bl = lds + MM * LD;  // Rbar, later W
    double *Tl = lds + 2 * MM * LD;  // M
    const bool in = c < MM;
    // row c of M = R Rbar^T: M[c][j] = sum_l R[c][l] Rbar[j][l]
    double mrow[MM];
    {
        double rrow[MM];
#pragma unroll
        for (int l = 0; l < MM; ++l) rrow[l] = in ? Rl[c * LD + l] : 0.0;
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int l = 0; l < MM; ++l) acc = fma(rrow[l], Bl[j * LD + l], acc);
            mrow[j] = acc;
        }
    }
    wave_lds_sync();
    if (in) {
#pragma unroll
        for (int j = 0; j < MM; ++j) Tl[c * LD + j] = mrow[j];
    }
    wave_lds_sync();
    // C = copyltu(M) is symmetric; lane c builds row (= column) c, then column c of
    // W = R^-1 C by back substitution
    double w[MM];
    {
        double crow[MM];
#pragma unroll
        for (int j = 0; j < MM; ++j) crow[j] = (j <= c) ? mrow[j] : (in ? Tl[j * LD + c] : 0.0);
#pragma unroll
        for (int i = MM - 1; i >= 0; --i) {
            double acc = crow[i];
#pragma unroll
            for (int l = i + 1; l < MM; ++l) acc = fma(-Rl[i * LD + l], w[l], acc);
            w[i] = acc / Rl[i * LD + i];
        }
    }
    wave_lds_sync();
    if (in) {
#pragma unroll
        for (int i = 0; i < MM; ++i) Bl[i * LD + c] = w[i];
    }
    wave_lds_sync();
    // row c of V solves R x = (row c of W)^T
#pragma unroll
    for (int l = 0; l < MM; ++l) w[l] = in ? Bl[c * LD + l] : 0.0;
#pragma unroll
    for (int p = MM - 1; p >= 0; --p) {
        double acc = w[p];
#pragma unroll
        for (int l = p + 1; l < MM; ++l) acc = fma(-Rl[p * LD + l], vrow[l], acc);
        vrow[p] = acc / Rl[p * LD + p];
    }
    wave_lds_sync();
}

}  // namespace gs
