// Regression coefficients of every family from the walk's R (gs_score_beta).
//
// Sec. 1.1: once the QRD of [X_S, x_c] is known, the regression of x_c on X_S is
// solved by back-substitution on its R, O(|S|^2).  Every R the walk visits is the QRD
// of its column ordering, so each family it emits ("prefix -> later column", Sec. 2)
// gets its coefficients from the leading block of that R:
//     R[P][P] beta = R[P][c],   P = the prefix positions,
// with the rows of the front variables included (the score walk drops them because no
// RSS needs them; the coefficients of a front parent do).
//
// One 32-lane group per segment (the split of Sec. 6, segment s: variable k + b in
// front when bit b of s is set), FP64.  The group first forms the segment's full R
// from R0 (Householder QR of R0 D P, D the power-of-two column equilibration), keeps it
// in LDS as R[row][lane] (lane = the variable's slot in the segment's initial
// ordering), then walks the paper's sequence Upsilon(k) on the walked block, swapping
// positions and restoring the triangle with one Givens step per swap.  After the start
// and after every swap, each child lane back-substitutes its own column against the
// prefix block and writes its coefficient row (zeros for non-parents); coefficients of
// the equilibrated data are turned back into those of X by exact powers of two.
#include <hip/hip_runtime.h>

#include <cmath>

#include "gs_internal.hpp"
#include "segment_qr.hpp"

namespace gs {

template <int MM>
__global__ __launch_bounds__(32) void beta_walk_kernel(const double *__restrict__ R0,
                                                       const ColStats *__restrict__ stats, int m,
                                                       int k, const int8_t *__restrict__ ups,
                                                       int64_t nups, double *__restrict__ out) {
    __shared__ double Rl[MM][MM];
    __shared__ double pc[MM];
    __shared__ double B[MM][MM + 1];  // per child lane: its coefficients by prefix position
    __shared__ int order[MM];         // lane holding the variable at each position
    __shared__ int lab[MM];           // variable label of each lane
    const int lane = threadIdx.x;     // 0..31
    const uint64_t s = blockIdx.x;
    const int d = __popcll((unsigned long long)s);
    const int label = segment_label(s, lane, m, k, k);  // walked block: labels 0..k-1
    double col[MM];
    segment_qr<MM>(R0, stats->scale, m, label, lane, col, pc, m);
    if (lane < MM) {
#pragma unroll
        for (int i = 0; i < MM; ++i) Rl[i][lane] = col[i];
        order[lane] = lane;
        lab[lane] = label;
    }
    int pos = lane;  // position of this lane's variable
    const int ec = label >= 0 ? stats->exp2[label] : 0;
    wave_lds_sync();

    // families "first p positions -> this lane's variable" for this lane, if it is later
    auto emit = [&](int p) {
        if (lane >= m || pos < p) return;
        uint64_t S = 0;
        for (int q = p - 1; q >= 0; --q) {
            const int lq = order[q];
            double acc = Rl[q][lane];
            for (int q2 = q + 1; q2 < p; ++q2) acc = fma(-Rl[q][order[q2]], B[lane][q2], acc);
            B[lane][q] = acc / Rl[q][lq];
            S |= uint64_t(1) << lab[lq];
        }
        const uint64_t low = S & ((uint64_t(1) << label) - 1);
        const uint64_t high = (S >> (label + 1)) << label;
        double *row = out + ((int64_t(label) << (m - 1)) + int64_t(low | high)) * m;
        for (int v = 0; v < m; ++v) row[v] = 0.0;
        for (int q = 0; q < p; ++q) {
            const int v = lab[order[q]];
            row[v] = ldexp(B[lane][q], ec - stats->exp2[v]);
        }
    };
    for (int p = d; p <= d + k && p < m; ++p) emit(p);
    for (int64_t t = 0; t < nups; ++t) {
        const int a = d + int(ups[t]);  // swap positions a and a + 1
        const int u = order[a], v = order[a + 1];
        wave_lds_sync();
        if (lane == 0) {
            order[a] = v;
            order[a + 1] = u;
        }
        pos = lane == u ? a + 1 : (lane == v ? a : pos);
        // Givens step on rows a, a + 1 with the pivot column v (reflector form, new
        // diagonal rho >= 0; rho = 0 only for a rank-deficient prefix: c = 1, s = 0)
        const double x = Rl[a][v], y = Rl[a + 1][v];
        const double rho = sqrt(fma(x, x, y * y));
        const double cs = rho > 0.0 ? x / rho : 1.0, sn = rho > 0.0 ? y / rho : 0.0;
        wave_lds_sync();
        if (lane < m) {
            const double r1 = Rl[a][lane], r2 = Rl[a + 1][lane];
            Rl[a][lane] = fma(cs, r1, sn * r2);
            Rl[a + 1][lane] = lane == v ? 0.0 : fma(sn, r1, -cs * r2);
        }
        wave_lds_sync();
        emit(a + 1);
    }
}

hipError_t launch_beta_walk(const double *R0, const ColStats *stats, int m, int k,
                            const int8_t *ups, int64_t nups, double *out, hipStream_t s) {
    const dim3 grid(unsigned(int64_t(1) << (m - k))), block(32);
    switch ((m + 3) / 4 * 4) {
#define GS_BETA_CASE(MMV)                                                                     \
    case MMV:                                                                                 \
        hipLaunchKernelGGL((beta_walk_kernel<MMV>), grid, block, 0, s, R0, stats, m, k, ups,  \
                           nups, out);                                                        \
        break;
        GS_BETA_CASE(4)
        GS_BETA_CASE(8)
        GS_BETA_CASE(12)
        GS_BETA_CASE(16)
        GS_BETA_CASE(20)
        GS_BETA_CASE(24)
#undef GS_BETA_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gs
