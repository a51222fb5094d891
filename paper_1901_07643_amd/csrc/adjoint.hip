// Reverse mode of the whole path: d(loss)/dX from d(loss)/d(score) of every family.
//
// The paper only computes scores; the adjoint is this library's.  It runs the chain
// X -> R0 -> segment anchors -> walk -> RSS -> score backwards:
//   1. walk_adjoint_kernel: per segment, the walk is replayed to its end (or, for long
//      walks, its end state is formed directly as the R of the final ordering, one QR
//      per segment like the anchors), then undone step by step.  Every Givens step is a
//      reflector, its own inverse, and the
//      rotation of a step is recovered from the matrix after the step: the column that
//      moved from position j to j+1 holds (c x, s x) there, x > 0 its old diagonal
//      (anchors have a non-negative diagonal and every step keeps it so).  Nothing is
//      stored per step.  Adjoints of the RSS sums are kept as lazy suffix-sum
//      accumulators, so each undone step costs O(1) per column.  Output: the adjoint
//      of the segment's anchor rows and of its back-row tails (FP64).
//   2. anchor_adjoint_kernel: the reverse rule of the anchor QR A = R0 P -> R
//      (Abar = A R^-1 copyltu(R Rbar^T) R^-T) gives each segment's V in label order;
//      their sum B gives R0bar = R0 B.
//   3. final_k_kernel: the reverse rule of X = Q0 R0 with R0bar restricted to the upper
//      triangle gives Xbar = X K, K = R0^-1 copyltu(R0 R0bar^T) R0^-T.
//   4. dx_kernel: dX = X K.
// Like the forward path, every stage works on the column-equilibrated data X D
// (D = diag(2^-e_c) from the R0 pass): the walk adjoint sees RSS of X D, the anchor
// QRs are those of R0 D, and the chain ends with d/dX = (d/d(X D)) D, i.e.
// K = D K_D D.  For RSS scores the cotangent of RSS(c, S) of X D is dscores times
// 2^(2 e_c); it is carried as 2^(2 (e_c - E)), E = max e_c, and the common factor
// 2^(2E) is applied to dX at the very end, so no intermediate leaves the range.
// All reductions are in fixed order (no atomics): the result is bit-reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gs_internal.hpp"
#include "segment_qr.hpp"

namespace gs {

template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for_r(Fn &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_r<I + 1, N>(f);
    }
}

__device__ __forceinline__ float bcast_r(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bcast_r(double v, int addr) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, int(bits & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, int(bits >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

// Cross-lane moves for half_sum: DPP inside a 16-lane row (no LDS round trip), and
// ds_swizzle for lane ^ 16 inside each 32-lane group.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_r(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_r(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL>(int(b & 0xffffffffll)), hi = dpp_i<CTRL>(int(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}
constexpr int SWZ_XOR16 = 0x1F | (0x10 << 10);  // bitmask mode: and 0x1F, or 0, xor 0x10
__device__ __forceinline__ float xor16_r(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), SWZ_XOR16));
}
__device__ __forceinline__ double xor16_r(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_swizzle(int(b & 0xffffffffll), SWZ_XOR16);
    const int hi = __builtin_amdgcn_ds_swizzle(int(b >> 32), SWZ_XOR16);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

// Sums of a and of b over the 32 lanes of this half-wave (one segment), in every lane:
// pairs (lane ^ 1), quads (lane ^ 2), the two quads of each 8 (mirror inside 8), the two
// 8s of each row (mirror inside 16), then the two rows (lane ^ 16).  The two chains
// alternate, so each DPP add reads a value written two instructions earlier: a single
// chain needs wait states between a VALU write and a DPP read of it.
template <typename T>
__device__ __forceinline__ void half_sum2(T &a, T &b) {
    a += dpp_r<0xB1>(a);  // quad_perm [1, 0, 3, 2]
    b += dpp_r<0xB1>(b);
    a += dpp_r<0x4E>(a);  // quad_perm [2, 3, 0, 1]
    b += dpp_r<0x4E>(b);
    a += dpp_r<0x141>(a);  // row_half_mirror
    b += dpp_r<0x141>(b);
    a += dpp_r<0x140>(a);  // row_mirror
    b += dpp_r<0x140>(b);
    a += xor16_r(a);
    b += xor16_r(b);
}

// 1 / x: the hardware reciprocal in FP32 (within 1 ulp), a division in FP64
template <typename T>
__device__ __forceinline__ T recip_r(T x) {
    if constexpr (std::is_same_v<T, float>) return __builtin_amdgcn_rcpf(x);
    else return 1.0 / x;
}

// 1 / sqrt(x) for x >= the smallest normal (cs_from clamps): the hardware value refined by
// one Newton step in FP32, two in FP64 (as in the forward walks)
template <typename T>
__device__ __forceinline__ T rsq_r(T x) {
    if constexpr (std::is_same_v<T, float>) {
        const float y = __builtin_amdgcn_rsqf(x);
        const float r = fmaf(-x * y, y, 1.0f);
        return fmaf(0.5f * y, r, y);
    } else {
        return rsq_newton(x);
    }
}

template <typename T>
__device__ __forceinline__ void cs_from(T a, T b, T &c, T &s) {
    const T rr = a * a + b * b;
    const T tiny = std::is_same_v<T, float> ? T(1.17549435e-38f) : T(2.2250738585072014e-308);
    const T r = rsq_r(rr > tiny ? rr : tiny);
    c = rr > T(0) ? a * r : T(1);
    s = b * r;
}

struct AdjArgs {
    int m, k, q;
    int64_t nseg, nsub;
    double n;
    int bic;
    const ColStats *stats;
};

// E = the largest equilibration exponent of the dataset (RSS cotangents are carried
// relative to 2^(2E))
__device__ __forceinline__ int max_exp2(const ColStats *st, int m) {
    int e = st->exp2[0];
    for (int c = 1; c < m; ++c) e = max(e, st->exp2[c]);
    return e;
}

constexpr int ADJ_HALVES = 4;  // segments per 128-thread workgroup

// NS consecutive cotangents of one table line with 16-byte loads.  A line starts at a
// multiple of NS entries of the 16-byte aligned table, so the loads are aligned.
template <typename T, int NS>
__device__ __forceinline__ void load_line(const T *__restrict__ src, T (&v)[NS]) {
    constexpr int VW = 16 / int(sizeof(T));
    if constexpr (NS % VW == 0) {
        typedef T VT __attribute__((ext_vector_type(VW)));
        const VT *p = reinterpret_cast<const VT *>(src);
        static_for_r<0, NS / VW>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            const VT w = p[i];
            static_for_r<0, VW>([&](auto ec) {
                constexpr int e = decltype(ec)::value;
                v[i * VW + e] = w[e];
            });
        });
    } else {
#pragma unroll
        for (int U = 0; U < NS; ++U) v[U] = src[U];
    }
}

// Forward Givens step on rows (x, y) with pivot lane address paddr (the column moving
// from j+1 to j); the pivot's new row-(j+1) entry is set to exactly zero.
template <typename T>
__device__ __forceinline__ void fwd_step(T &x, T &y, int paddr, bool is_piv) {
    T c, s;
    cs_from(bcast_r(x, paddr), bcast_r(y, paddr), c, s);
    const T nx = c * x + s * y;
    const T ny = s * x - c * y;
    x = nx;
    y = is_piv ? T(0) : ny;
}

// Undo one forward step and carry its adjoint back.  On entry (x, y) are rows j, j+1
// after the step and (xb, yb) their adjoints; is_piv marks the pivot column's lane (its
// row-j entry after the step is rho), maddr / is_mov the column that moved from j to
// j+1.  On return: rows and adjoints before the step.
template <typename T>
__device__ __forceinline__ void rev_step(T &x, T &y, T &xb, T &yb, int maddr, bool is_piv,
                                         bool is_mov) {
    T c, s;
    cs_from(bcast_r(x, maddr), bcast_r(y, maddr), c, s);
    const T xa = x, ya = y;
    const T xba = xb, yba = is_piv ? T(0) : yb;  // the pivot's new row-(j+1) entry is a constant
    const T x0 = c * xa + s * ya;
    const T y0 = is_mov ? T(0) : s * xa - c * ya;
    T xb0 = c * xba + s * yba;
    T yb0 = s * xba - c * yba;
    T cb = xba * x0 - yba * y0;
    T sb = xba * y0 + yba * x0;
    half_sum2(cb, sb);
    // the pivot lane carries the adjoints of c and s (through rho) back to its rows; its
    // own row-j entry after the step is rho
    const T rinv = (is_piv && xa != T(0)) ? recip_r(xa) : T(0);
    const T t = (cb * s - sb * c) * rinv;
    xb0 += s * t;
    yb0 -= c * t;
    x = x0;
    y = y0;
    xb = xb0;
    yb = yb0;
}

// FP32 with inner block 5: 128 VGPRs, 4 waves per SIMD, so that the 2^(m-k) / 2 waves of
// the headline split (k = 13) are resident at once
template <typename T, int KS>
constexpr int kAdjMinWaves = (std::is_same_v<T, float> && KS == 5) ? 4 : 1;

template <typename T, int KS>
__global__ __launch_bounds__(32 * ADJ_HALVES)
__attribute__((amdgpu_waves_per_eu(kAdjMinWaves<T, KS>, 8))) void walk_adjoint_kernel(
    const T *__restrict__ anchor, const T *__restrict__ tail, const T *__restrict__ anchor_end,
    int z_end, const uint32_t *__restrict__ prog, const T *__restrict__ dscores,
    double *__restrict__ anchorbar, double *__restrict__ tailbar, AdjArgs a) {
    constexpr int N = InnerProgram<KS>::N;
    constexpr int NS = 1 << KS;
    __shared__ T Lrows[ADJ_HALVES][Q_MAX][32];
    __shared__ T Lbars[ADJ_HALVES][Q_MAX][32];
    const int hw = threadIdx.x >> 5;
    const int lane = threadIdx.x & 31;
    const int64_t seg = int64_t(blockIdx.x) * ADJ_HALVES + hw;
    const bool ok = seg < a.nseg;
    const int m = a.m, k = a.k, q = a.q, nout = m - k;
    const int base = (threadIdx.x & 32) * 4;  // ds_bpermute address of this half's lane 0
    T(*L)[32] = Lrows[hw];
    T(*Lb)[32] = Lbars[hw];

    const uint64_t scode = ok ? uint64_t(seg) : 0;
    int label = -1, cls = 0;
    if (lane < KS) {
        label = lane;
        cls = 1;
    } else if (lane < k) {
        label = lane;
        cls = 2;
    } else {
        int cnt = 0;
        for (int b = 0; b < nout; ++b)
            if (!((scode >> b) & 1)) {
                if (cnt == lane - k) {
                    label = k + b;
                    cls = 3;
                }
                ++cnt;
            }
    }
    if (!ok) cls = 0;
    const uint64_t Fbits = scode << k;

    // lanes past the segment's k + b columns hold no column (the anchor buffer is not
    // written there): they must carry zeros, since the rotation adjoints sum over lanes
    const bool col_ok = cls != 0;
    // the walk's state: at its start (anchor, inner block behind all q middle rows), or
    // with anchor_end at its end (inner block from middle row z_end on), where the
    // reverse walk begins without a replay
    const T *an = (anchor_end ? anchor_end : anchor) + int64_t(ok ? seg : 0) * k * 32 + lane;
    int z = anchor_end ? z_end : q;
    T I[KS], Ib[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) {
        I[i] = col_ok ? an[(z + i) * 32] : T(0);
        Ib[i] = T(0);
    }
    for (int p = 0; p < q; ++p) {
        L[p][lane] = col_ok ? an[(p < z ? p : p + KS) * 32] : T(0);
        Lb[p][lane] = T(0);
    }
    const T tl = col_ok ? tail[int64_t(seg) * 32 + lane] : T(0);
    T tlb = T(0);
    const T nn = T(a.n);
    // RSS scores: d(RSS of X)/d(RSS of X D) = 2^(2 e_c), carried relative to 2^(2E)
    const T gscale = (a.bic || label < 0)
                         ? T(1)
                         : T(ldexp(1.0, 2 * (a.stats->exp2[label] - max_exp2(a.stats, m))));

    // 1. replay the walk to its end (rotations only), unless it starts there
    auto forward_sub = [&](auto dirc, uint32_t w1) {
        constexpr bool FWD = decltype(dirc)::value;
        constexpr auto &ord = FWD ? kInner<KS>.order_f : kInner<KS>.order_r;
        if (w1 & SubWord::kHasTransition) {
            if (w1 & SubWord::kHasMid) {
                const int j = int((w1 >> 2) & 31), piv = int((w1 >> 8) & 31);
                T x = L[j][lane], y = L[j + 1][lane];
                fwd_step(x, y, base + piv * 4, lane == piv);
                L[j][lane] = x;
                L[j + 1][lane] = y;
            }
            const int v = int((w1 >> 16) & 31);
            if (w1 & SubWord::kCrossLeft) {
                T carry = L[z][lane];
                static_for_r<0, KS>([&](auto ic) {
                    constexpr int i = KS - 1 - decltype(ic)::value;
                    T x = I[i], y = carry;
                    fwd_step(x, y, base + v * 4, lane == v);
                    carry = x;
                    I[i] = y;
                });
                L[z][lane] = carry;
                ++z;
            } else {
                T carry = L[z - 1][lane];
                static_for_r<0, KS>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    T x = carry, y = I[i];
                    fwd_step(x, y, base + ord[i] * 4, lane == ord[i]);
                    I[i] = x;
                    carry = y;
                });
                L[z - 1][lane] = carry;
                --z;
            }
        }
        static_for_r<0, N>([&](auto sc) {
            constexpr int st = decltype(sc)::value;
            constexpr int J = FWD ? kInner<KS>.j_f[st] : kInner<KS>.j_r[st];
            constexpr int PV = FWD ? kInner<KS>.piv_f[st] : kInner<KS>.piv_r[st];
            fwd_step(I[J], I[J + 1], base + PV * 4, lane == PV);
        });
    };
    if (!anchor_end) {
        for (int64_t t = 0; t < a.nsub; ++t) {
            const uint32_t w1 = prog[2 * t + 1];
            if ((t & 1) == 0) forward_sub(std::true_type{}, w1);
            else forward_sub(std::false_type{}, w1);
        }
    }

    // 2. undo it, sub-walk by sub-walk
    auto reverse_sub = [&](auto dirc, uint32_t w0, uint32_t w1) {
        constexpr bool FWD = decltype(dirc)::value;
        constexpr auto &ord = FWD ? kInner<KS>.order_f : kInner<KS>.order_r;
        const uint32_t omask = w0 & 0xFFFFu;
        // this lane's cotangents for the sub-walk's 2^KS parent sets (slot = inner subset)
        T gl[NS];
        const uint64_t Shi = Fbits | (uint64_t(omask) << KS);
        const int64_t cbase = int64_t(label) << (m - 1);
        const bool child = cls == 1 || cls == 3 || (cls == 2 && !((omask >> (lane - KS)) & 1u));
        int64_t lbase = 0;
        if (cls == 1) {
            lbase = cbase + int64_t(Shi >> 1);
        } else if (child) {
            const uint64_t lo = Shi & ((uint64_t(1) << label) - 1);
            const uint64_t hi = (Shi >> (label + 1)) << label;
            lbase = cbase + int64_t(lo | hi);
        }
#pragma unroll
        for (int U = 0; U < NS; ++U) gl[U] = T(0);
        if (cls == 1) {
            // inner child: the entries without its own bit, gathered
#pragma unroll
            for (int U = 0; U < NS; ++U) {
                if (!((U >> lane) & 1)) {
                    const int lowm = (1 << lane) - 1;
                    gl[U] = dscores[lbase + ((U & lowm) | ((U >> (lane + 1)) << lane))];
                }
            }
        } else if (child) {
            load_line<T, NS>(dscores + lbase, gl);  // its whole line
        }
        T bsum = tl;
        for (int p = q - 1; p >= z; --p) bsum = L[p][lane] * L[p][lane] + bsum;
        T sfx[KS + 1], Sb[KS + 1];
        sfx[KS] = bsum;
#pragma unroll
        for (int i = KS - 1; i >= 0; --i) sfx[i] = I[i] * I[i] + sfx[i + 1];
#pragma unroll
        for (int i = 0; i <= KS; ++i) Sb[i] = T(0);
        // dBIC/dRSS = n / RSS; lanes that are not children carry g = 0 (and possibly a
        // zero RSS), which must stay 0: a NaN would reach every lane through the sums
        // of the rotation adjoints
        auto gbar = [&](T rss, T g) -> T {
            return (a.bic && g != T(0)) ? g * nn * recip_r(rss) : g * gscale;
        };
        static_for_r<0, N>([&](auto sc) {
            constexpr int st = N - 1 - decltype(sc)::value;
            constexpr int J = FWD ? kInner<KS>.j_f[st] : kInner<KS>.j_r[st];
            constexpr int PV = FWD ? kInner<KS>.piv_f[st] : kInner<KS>.piv_r[st];
            constexpr int MV = FWD ? kInner<KS>.mov_f[st] : kInner<KS>.mov_r[st];
            constexpr int U = FWD ? kInner<KS>.mask_f[st] : kInner<KS>.mask_r[st];
            // the family emitted after this step: RSS = suffix sum from row J+1
            Sb[J + 1] += gbar(sfx[J + 1], gl[U]);
            // the step changes row J+1's suffix sum: turn its accumulator into row terms
            Ib[J + 1] += T(2) * I[J + 1] * Sb[J + 1];
            Sb[J + 2] += Sb[J + 1];
            Sb[J + 1] = T(0);
            rev_step(I[J], I[J + 1], Ib[J], Ib[J + 1], base + MV * 4, lane == PV,
                     lane == MV);
            sfx[J + 1] = I[J + 1] * I[J + 1] + sfx[J + 2];
        });
        static_for_r<0, KS + 1>([&](auto pc) {
            constexpr int pl = decltype(pc)::value;
            constexpr int U = FWD ? kInner<KS>.init_f[pl] : kInner<KS>.init_r[pl];
            Sb[pl] += gbar(sfx[pl], gl[U]);
        });
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < KS; ++i) {
            acc += Sb[i];
            Ib[i] += T(2) * I[i] * acc;
        }
        acc += Sb[KS];
        for (int p = z; p < q; ++p) Lb[p][lane] += T(2) * L[p][lane] * acc;
        tlb += acc;

        if (w1 & SubWord::kHasTransition) {
            const int v = int((w1 >> 16) & 31);
            if (w1 & SubWord::kCrossLeft) {
                --z;
                T carry = L[z][lane], carryb = Lb[z][lane];
                static_for_r<0, KS>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    T x = carry, y = I[i], xb = carryb, yb = Ib[i];
                    rev_step(x, y, xb, yb, base + ord[i] * 4, lane == v,
                             lane == ord[i]);
                    I[i] = x;
                    Ib[i] = xb;
                    carry = y;
                    carryb = yb;
                });
                L[z][lane] = carry;
                Lb[z][lane] = carryb;
            } else {
                T carry = L[z][lane], carryb = Lb[z][lane];
                static_for_r<0, KS>([&](auto ic) {
                    constexpr int i = KS - 1 - decltype(ic)::value;
                    T x = I[i], y = carry, xb = Ib[i], yb = carryb;
                    rev_step(x, y, xb, yb, base + v * 4, lane == ord[i],
                             lane == v);
                    carry = x;
                    carryb = xb;
                    I[i] = y;
                    Ib[i] = yb;
                });
                L[z][lane] = carry;
                Lb[z][lane] = carryb;
                ++z;
            }
            if (w1 & SubWord::kHasMid) {
                const int j = int((w1 >> 2) & 31), piv = int((w1 >> 8) & 31);
                const int mv = int((w0 >> 21) & 31);
                T x = L[j][lane], y = L[j + 1][lane], xb = Lb[j][lane], yb = Lb[j + 1][lane];
                rev_step(x, y, xb, yb, base + mv * 4, lane == piv, lane == mv);
                L[j][lane] = x;
                L[j + 1][lane] = y;
                Lb[j][lane] = xb;
                Lb[j + 1][lane] = yb;
            }
        }
    };
    for (int64_t t = a.nsub - 1; t >= 0; --t) {
        const uint32_t w0 = prog[2 * t], w1 = prog[2 * t + 1];
        if ((t & 1) == 0) reverse_sub(std::true_type{}, w0, w1);
        else reverse_sub(std::false_type{}, w0, w1);
    }

    if (!ok) return;
    double *ab = anchorbar + int64_t(seg) * k * 32 + lane;
    for (int p = 0; p < q; ++p) ab[p * 32] = double(Lb[p][lane]);
#pragma unroll
    for (int i = 0; i < KS; ++i) ab[(q + i) * 32] = double(Ib[i]);
    tailbar[int64_t(seg) * 32 + lane] = double(tlb);
}

// Per segment: V = R^-1 copyltu(R Rbar^T) R^-T of the anchor QR, written in label order.
template <int MM>
__global__ __launch_bounds__(64) void anchor_adjoint_kernel(const double *__restrict__ R0,
                                                            const ColStats *__restrict__ stats,
                                                            int m, int k, int ks, int64_t nseg,
                                                            const double *__restrict__ anchorbar,
                                                            const double *__restrict__ tailbar,
                                                            double *__restrict__ vout) {
    constexpr int LD = MM + 1;
    __shared__ double pcol[2][MM];
    __shared__ double work[2][3 * MM * LD];
    __shared__ int labels[2][32];
    const int hw = threadIdx.x >> 5;
    const int c = threadIdx.x & 31;
    const int64_t seg = int64_t(blockIdx.x) * 2 + hw;
    const bool ok = seg < nseg;
    const uint64_t s = ok ? uint64_t(seg) : 0;
    const int d = __popcll((unsigned long long)s);
    const int label = ok ? segment_label(s, c, m, k, ks) : -1;
    double col[MM];
    segment_qr<MM>(R0, stats->scale, m, label, c, col, pcol[hw], m);
    double rbar[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) rbar[i] = 0.0;
    if (ok && c >= d && c < m) {
        const int l = label < k ? label : c - d;
        const double *abp = anchorbar + seg * int64_t(k) * 32 + l;
        const double tb = tailbar[seg * 32 + l];
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            const int r = i - d;
            if (i <= c) {
                if (r >= 0 && r < k) rbar[i] = abp[r * 32];
                else if (r >= k && i < m && label >= k) rbar[i] = 2.0 * tb * col[i];
            }
        }
    }
    labels[hw][c] = label;
    qr_adj_store<MM>(col, rbar, c, work[hw]);
    double vrow[MM];
    qr_adjoint_core<MM>(c, work[hw], vrow);
    if (!ok || c >= m) return;
    double *vo = vout + seg * int64_t(m) * m + int64_t(label) * m;
#pragma unroll
    for (int p = 0; p < MM; ++p)
        if (p < m) vo[labels[hw][p]] = vrow[p];
}

// partial[ch][e] = sum of vout[seg][e] over the segments of chunk ch (fixed order)
// Partial sums of the per-segment V blocks: chunk ch (of VSUM_CHUNKS) adds its
// consecutive segments for one matrix element per thread, in segment order.
constexpr int VSUM_CHUNKS = 64;
__global__ __launch_bounds__(256) void sum_v_kernel(const double *__restrict__ vout, int64_t nseg,
                                                    int64_t per_chunk, int mm,
                                                    double *__restrict__ partial) {
    const int64_t ch = blockIdx.x;
    const int e = int(blockIdx.y) * 256 + int(threadIdx.x);
    if (e >= mm) return;
    const int64_t s0 = ch * per_chunk, s1 = min(nseg, s0 + per_chunk);
    double acc = 0.0;
#pragma unroll 8
    for (int64_t sg = s0; sg < s1; ++sg) acc += vout[sg * mm + e];
    partial[ch * mm + e] = acc;
}

// B = sum of the partials; R0bar = triu(R0 B); K = R0^-1 copyltu(R0 R0bar^T) R0^-T.
constexpr int FINALK_THREADS = 256;

template <int MM>
__global__ __launch_bounds__(FINALK_THREADS) void final_k_kernel(const double *__restrict__ R0,
                                                     const ColStats *__restrict__ stats, int m,
                                                     const double *__restrict__ partial,
                                                     int64_t nchunks, double *__restrict__ Bout,
                                                     double *__restrict__ K) {
    constexpr int LD = MM + 1;
    __shared__ double Bs[32 * 32];
    __shared__ double R0s[32 * 32];  // R0 D
    __shared__ double work[3 * MM * LD];
    const int c = threadIdx.x;
    const int mm = m * m;
    for (int e = c; e < mm; e += FINALK_THREADS) R0s[e] = R0[e] * stats->scale[e % m];
    // one entry of B per thread; the chunk loop is unrolled so that its loads are in
    // flight together (the additions keep their fixed order)
    for (int e = c; e < mm; e += FINALK_THREADS) {
        double acc = 0.0;
#pragma unroll 16
        for (int64_t ch = 0; ch < nchunks; ++ch) acc += partial[ch * mm + e];
        Bs[e] = acc;
        Bout[e] = acc;
    }
    __syncthreads();
    if (c >= 32) return;
    double col[MM], rbar[MM];
#pragma unroll
    for (int i = 0; i < MM; ++i) {
        col[i] = (c < m) ? (i < m ? R0s[i * m + c] : 0.0) : (i == c ? 1.0 : 0.0);
        double acc = 0.0;
        if (c < m && i < m && i <= c)
            for (int l = i; l < m; ++l) acc = fma(R0s[i * m + l], Bs[l * m + c], acc);
        rbar[i] = acc;
    }
    qr_adj_store<MM>(col, rbar, c, work);
    double vrow[MM];
    qr_adjoint_core<MM>(c, work, vrow);
    if (c < m)
        for (int p = 0; p < m; ++p) K[c * m + p] = vrow[p];
}

// dX = (X D) K_D D 2^(2E)  (K_D of the equilibrated problem, D = diag(2^-exp2); X: n x m,
// row stride ldx; dX: row stride lddx; 2E only for RSS scores)
__global__ __launch_bounds__(256) void dx_kernel(const double *__restrict__ X, int64_t n, int m,
                                                 int64_t ldx, const double *__restrict__ K,
                                                 const ColStats *__restrict__ stats, int bic,
                                                 double *__restrict__ dX, int64_t lddx) {
    __shared__ double Ks[32 * 32];
    __shared__ int ex[32];
    __shared__ int gexp;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) Ks[e] = K[e];
    if (threadIdx.x < m) ex[threadIdx.x] = stats->exp2[threadIdx.x];
    if (threadIdx.x == 0) gexp = bic ? 0 : 2 * max_exp2(stats, m);
    __syncthreads();
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * m) return;
    const int64_t r = idx / m;
    const int j = int(idx - r * m);
    double acc = 0.0;
    for (int i = 0; i < m; ++i) acc = fma(ldexp(X[r * ldx + i], -ex[i]), Ks[i * m + j], acc);
    dX[r * lddx + j] = ldexp(acc, gexp - ex[j]);
}

template <typename T>
hipError_t launch_walk_adjoint(const gs_plan_s *p, const T *anchor, const T *tail,
                               const T *anchor_end, const T *dscores, double *anchorbar,
                               double *tailbar, int64_t n, bool bic, hipStream_t s) {
    AdjArgs a;
    a.m = p->m;
    a.k = p->k;
    a.q = p->q;
    a.nseg = p->nseg;
    a.nsub = p->nsub;
    a.n = double(n);
    a.bic = bic ? 1 : 0;
    a.stats = p->d_stats;
    const dim3 grid(unsigned((p->nseg + ADJ_HALVES - 1) / ADJ_HALVES)), block(32 * ADJ_HALVES);
    switch (p->ks) {
#define GS_ADJ_CASE(KSV)                                                                     \
    case KSV:                                                                                \
        hipLaunchKernelGGL((walk_adjoint_kernel<T, KSV>), grid, block, 0, s, anchor, tail,   \
                           anchor_end, p->end.z, p->d_prog, dscores, anchorbar, tailbar, a); \
        break;
        GS_ADJ_CASE(1)
        GS_ADJ_CASE(2)
        GS_ADJ_CASE(3)
        GS_ADJ_CASE(4)
        GS_ADJ_CASE(5)
        GS_ADJ_CASE(6)
#undef GS_ADJ_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_walk_adjoint<float>(const gs_plan_s *, const float *, const float *,
                                               const float *, const float *, double *, double *,
                                               int64_t, bool, hipStream_t);
template hipError_t launch_walk_adjoint<double>(const gs_plan_s *, const double *, const double *,
                                                const double *, const double *, double *, double *,
                                                int64_t, bool, hipStream_t);

int64_t adjoint_partial_chunks(int64_t nseg) { return nseg < VSUM_CHUNKS ? nseg : VSUM_CHUNKS; }

hipError_t launch_qr_adjoint_chain(const gs_plan_s *p, const double *R0, const ColStats *stats,
                                   bool bic, const double *anchorbar,
                                   const double *tailbar, double *vout, double *partial, double *B,
                                   double *K, const double *X, int64_t n, int64_t ldx, double *dX,
                                   int64_t lddx, hipStream_t s) {
    const int m = p->m;
    // columns padded to a multiple of 4; above 24 to 32: the instance for 28 columns
    // exceeds the register file and spills to scratch, the one for 32 does not (the
    // one for 24 spills less and is still faster than padding to 32)
    const int mm = m > 24 ? 32 : (m + 3) / 4 * 4;
    const dim3 ag(unsigned((p->nseg + 1) / 2));
    switch (mm) {
#define GS_AADJ_CASE(MMV)                                                                        \
    case MMV:                                                                                    \
        hipLaunchKernelGGL((anchor_adjoint_kernel<MMV>), ag, dim3(64), 0, s, R0, stats, m, p->k, \
                           p->ks, p->nseg, anchorbar, tailbar, vout);                            \
        break;
        GS_AADJ_CASE(4)
        GS_AADJ_CASE(8)
        GS_AADJ_CASE(12)
        GS_AADJ_CASE(16)
        GS_AADJ_CASE(20)
        GS_AADJ_CASE(24)
        GS_AADJ_CASE(32)
#undef GS_AADJ_CASE
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nch = adjoint_partial_chunks(p->nseg);
    const int64_t per_chunk = (p->nseg + nch - 1) / nch;
    hipLaunchKernelGGL(sum_v_kernel, dim3(unsigned(nch), unsigned((m * m + 255) / 256)), dim3(256), 0,
                       s, vout, p->nseg, per_chunk, m * m, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    switch (mm) {
#define GS_FK_CASE(MMV)                                                                       \
    case MMV:                                                                                 \
        hipLaunchKernelGGL((final_k_kernel<MMV>), dim3(1), dim3(FINALK_THREADS), 0, s, R0, stats, \
                           m,                                                                 \
                           partial, nch,                                                      \
                           B, K);                                                             \
        break;
        GS_FK_CASE(4)
        GS_FK_CASE(8)
        GS_FK_CASE(12)
        GS_FK_CASE(16)
        GS_FK_CASE(20)
        GS_FK_CASE(24)
        GS_FK_CASE(32)
#undef GS_FK_CASE
        default: return hipErrorInvalidValue;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t tot = n * m;
    hipLaunchKernelGGL(dx_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, X, n, m, ldx,
                       K, stats, bic ? 1 : 0, dX, lddx);
    return hipGetLastError();
}

}  // namespace gs
