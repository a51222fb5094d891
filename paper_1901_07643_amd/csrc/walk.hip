// The walk: adjacent column swaps with one Givens retriangularisation each
// (Sec. 1.3), along the shortest sequence of orderings (Sec. 3-4), split into
// independent segments (Sec. 6), with every visited R turned into RSS and BIC
// values of the families it solves (Sec. 2) and written to the score table.
//
// Mapping to the GPU: segments are packed side by side into 64-lane waves (a
// segment of k walked and b back variables takes k + b lanes); every segment
// runs the same program, so a wave costs the same whatever it holds.
//   - each lane holds the column of one variable of its segment (slots 0..ks-1
//     the inner block, ks..k-1 the middle variables, then the back variables).
//     A column swap is then only a relabelling; the Givens step mixes two rows in
//     every lane.
//   - the inner block's ks rows live in registers; the inner walk is unrolled at
//     compile time, so each row index is a constant.  The q middle rows live in
//     LDS, addressed at run time.
//   - the pivot column's two entries are broadcast to the segment's lanes with
//     ds_bpermute (each lane addresses its own segment's pivot slot).
//   - each inner walk fills one table line (2^ks consecutive entries) per child
//     column in registers; it is written out with 16-byte stores at its end.
//
// Givens step at rows (j, j+1) after exchanging the columns at positions j, j+1
// (Sec. 1.3): with a = r[j][piv], b = r[j+1][piv] of the new column at j+1... the
// pivot is the column that moves from j+1 to j, rho = sqrt(a^2 + b^2),
// c = a / rho, s = b / rho.  The rows become
//   r[j]   <- c r[j] + s r[j+1]
//   r[j+1] <- s r[j] - c r[j+1],
// the reflector form of the paper's rotation (it keeps the new diagonal entry
// rho positive and differs from the rotation only by the sign of row j+1, which
// no RSS depends on).  The pivot's new r[j+1] is set to exactly zero.  rho = 0
// (a rank-deficient prefix) uses c = 1, s = 0.
//
// RSS from R (the paper names the models each QRD solves but not the formula):
// for an ordering with variable c at position p, RSS(c | first i variables) is
// the sum of the squares of column c over rows i..p.  Per lane the kernels keep
// these suffix sums: after a swap at j only the one for row j+1 changes.
//
// The walk scores the column-equilibrated data X D (D = diag(2^-e_c), every column
// norm in [1/2, 1)): RSS(c, S) of X is the walk's value times 2^(2 e_c), exactly (an
// ldexp), and BIC gains the constant 2 e_c n ln 2 of the child.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "gs_internal.hpp"

namespace gs {

template <int I, int N, typename Fn>
__device__ __forceinline__ void static_for(Fn &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ float bcast(float v, int addr) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bcast(double v, int addr) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, int(bits & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, int(bits >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

template <typename T>
struct Arith;

template <>
struct Arith<float> {
    // hardware 1/sqrt plus one Newton step, so that c^2 + s^2 = 1 to rounding:
    // a biased normalisation error would scale the rows a little at every step
    static __device__ __forceinline__ float rsq(float x) {
        const float y = __builtin_amdgcn_rsqf(x);
        const float r = fmaf(-x * y, y, 1.0f);
        return fmaf(0.5f * y, r, y);
    }
    static __device__ __forceinline__ float tiny() { return 1.17549435e-38f; }
    static __device__ __forceinline__ float huge() { return 3.40282347e+38f; }
    static __device__ __forceinline__ float ldexp(float x, int e) {
        return __builtin_amdgcn_ldexpf(x, e);
    }
    // BIC from RSS/n: n ln(RSS/n) + cst = (n ln 2) log2(RSS/n) + cst
    static __device__ __forceinline__ float score(float rss, float nlog, float cst) {
        return fmaf(nlog, __builtin_amdgcn_logf(rss), cst);
    }
};

// ln x for the FP64 scores, branch-free: x = f 2^e with f in [sqrt(1/2), sqrt(2)), and
// ln f = 2 atanh(u) = 2 u (1 + u^2/3 + u^4/5 + ...), u = (f - 1) / (f + 1), |u| <= 0.1716,
// summed to u^19 (the rest is below 3e-16); e ln 2 uses ln 2 split into a 32-bit head,
// so that e times it is exact, and the remainder.  1 / (f + 1) is the hardware
// reciprocal refined by two Newton steps; a subnormal x is first scaled by 2^64.  x = 0
// (RSS of an exactly rank-deficient prefix) gives -inf, +inf gives +inf and NaN stays NaN.
__device__ __forceinline__ double ln_score(double x) {
    constexpr double LN2_HEAD = 0x1.62e42ffp-1;           // ln 2 to 32 bits
    constexpr double LN2_TAIL = -4.2009150726810846e-11;  // ln 2 - LN2_HEAD
    const bool sub = x < 2.2250738585072014e-308;
    const double xs = sub ? x * 0x1p64 : x;
    double f = __builtin_amdgcn_frexp_mant(xs);  // in [1/2, 1) for finite xs != 0
    int e = __builtin_amdgcn_frexp_exp(xs) - (sub ? 64 : 0);
    const bool lo = f < 0.70710678118654752;
    f = lo ? f + f : f;
    e = lo ? e - 1 : e;
    const double d = f + 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    const double u = (f - 1.0) * r;  // f - 1 is exact
    const double s = u * u;
    double p = 1.0 / 19;
    p = fma(p, s, 1.0 / 17);
    p = fma(p, s, 1.0 / 15);
    p = fma(p, s, 1.0 / 13);
    p = fma(p, s, 1.0 / 11);
    p = fma(p, s, 1.0 / 9);
    p = fma(p, s, 1.0 / 7);
    p = fma(p, s, 1.0 / 5);
    p = fma(p, s, 1.0 / 3);
    p = fma(p, s, 1.0);
    const double de = double(e);
    const double y = fma(de, LN2_HEAD, fma(de, LN2_TAIL, 2.0 * u * p));
    return x == 0.0 ? -__builtin_inf() : (x == __builtin_inf() ? x : y);
}

template <>
struct Arith<double> {
    // x >= the smallest normal here (the FP64 walk always takes the guarded path)
    static __device__ __forceinline__ double rsq(double x) { return rsq_newton(x); }
    static __device__ __forceinline__ double tiny() { return 2.2250738585072014e-308; }
    static __device__ __forceinline__ double huge() { return 1.7976931348623157e+308; }
    static __device__ __forceinline__ double ldexp(double x, int e) {
        return __builtin_amdgcn_ldexp(x, e);
    }
    static __device__ __forceinline__ double score(double rss, double nlog, double cst) {
        return fma(nlog, ln_score(rss), cst);
    }
};

// c, s of the step from the pivot's entries (a, b) at rows j, j+1.  With GUARD a
// zero pair (an exactly rank-deficient prefix) gives c = 1, s = 0; without it the
// caller knows that R0 has a clearly non-zero diagonal, so a^2 + b^2 > 0.
template <bool GUARD, typename T>
__device__ __forceinline__ void givens_cs(T a, T b, T &c, T &s) {
    const T rr = a * a + b * b;
    if constexpr (GUARD) {
        const T r = Arith<T>::rsq(rr > Arith<T>::tiny() ? rr : Arith<T>::tiny());
        c = rr > T(0) ? a * r : T(1);
        s = b * r;
    } else {
        const T r = Arith<T>::rsq(rr);
        c = a * r;
        s = b * r;
    }
}

struct WalkArgs {
    int m, k, q;
    int64_t nseg, nsub, nwaves;
    ReducePartials red;  // reduce modes only
    double row_scale;  // 1/sqrt(n) for BIC (the table then gets RSS/n inside the log), 1 for RSS
    double nlog;       // n ln 2 (FP32 path, log2 in hardware) or n (FP64 path)
    double lnn;        // ln n
    double nln2;       // n ln 2: BIC of X = BIC of X D + 2 e_c n ln 2
};

template <int CNT, typename T>
__device__ __forceinline__ void store_line(T *dst, const T *v) {
    constexpr int VE = 16 / int(sizeof(T));
    if constexpr (CNT % VE == 0) {
        using V = std::conditional_t<std::is_same_v<T, float>, float4, double2>;
        static_for<0, CNT / VE>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            V w;
            if constexpr (std::is_same_v<T, float>) {
                w.x = v[4 * i + 0];
                w.y = v[4 * i + 1];
                w.z = v[4 * i + 2];
                w.w = v[4 * i + 3];
            } else {
                w.x = v[2 * i + 0];
                w.y = v[2 * i + 1];
            }
            reinterpret_cast<V *>(dst)[i] = w;
        });
    } else {
        static_for<0, CNT>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            dst[i] = v[i];
        });
    }
}

// v_cndmask with a wave-uniform lane mask: lanes whose bit is set take `set`.
// Written as one instruction so that the compiler cannot turn a choice between two
// register-array elements into a run-time index into that array.
__device__ __forceinline__ float select_lanes(uint64_t mask, float set, float other) {
    float r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(other), "v"(set), "s"(mask));
    return r;
}
__device__ __forceinline__ double select_lanes(uint64_t mask, double set, double other) {
    const long long s = __double_as_longlong(set), o = __double_as_longlong(other);
    int lo, hi;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3"
                 : "=v"(lo) : "v"(int(o & 0xffffffffll)), "v"(int(s & 0xffffffffll)), "s"(mask));
    asm("v_cndmask_b32_e64 %0, %1, %2, %3"
                 : "=v"(hi) : "v"(int(o >> 32)), "v"(int(s >> 32)), "s"(mask));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                            (unsigned long long)(unsigned)lo));
}

// insert a zero bit at position c of i
__host__ __device__ constexpr int expand_bit(int i, int c) {
    return ((i >> c) << (c + 1)) | (i & ((1 << c) - 1));
}
// the value of expand_bit(i, c) shared by the most c in 0..ks-1 (ties: smallest c)
__host__ __device__ constexpr int common_expansion(int i, int ks) {
    int best = expand_bit(i, 0), most = 0;
    for (int c = 0; c < ks; ++c) {
        int n = 0;
        for (int d = 0; d < ks; ++d) n += expand_bit(i, d) == expand_bit(i, c);
        if (n > most) {
            most = n;
            best = expand_bit(i, c);
        }
    }
    return best;
}
// c is the smallest slot with its value of expand_bit(i, .)
__host__ __device__ constexpr bool first_expansion(int i, int c) {
    for (int d = 0; d < c; ++d)
        if (expand_bit(i, d) == expand_bit(i, c)) return false;
    return true;
}

// Table lines of the FP32 walk (inner block 5: 32 floats = 128 bytes) go out through
// an LDS stage: each lane puts its line (8 float4 chunks) and its destination into
// the stage, then each of 8 store instructions writes 8 whole lines, 8 consecutive
// lanes and 16 bytes per lane each.  A lane writing its own line spreads each store
// instruction over 64 cache lines, which HBM absorbs at little more than half the
// rate of whole lines.  Chunk c of lane o's line sits at Sg[64 c + (o ^ c)], so that
// both the writes (c fixed, o = lane) and the reads (8 lanes: one line, c = 0..7)
// hit distinct LDS banks.
constexpr int STAGE_LINES = 64, STAGE_CHUNKS = 8;
constexpr int STAGE_BYTES = STAGE_LINES * STAGE_CHUNKS * 16 + STAGE_LINES * 8;

typedef float native_float4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) native_float4 global_float4;

// 16-byte store through a global address-space pointer.  (A flat store would also
// count as an LDS operation, and every later wait for LDS would wait for it.)
__device__ __forceinline__ void global_store16(uint64_t dst, const float4 &v) {
    native_float4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *reinterpret_cast<global_float4 *>(dst) = w;
}

// Write-count mode of the walk (testing): every 4-byte table entry a store would write
// gets an atomic +1 instead, at the same address, through the same store path.
__device__ __forceinline__ void count16(uint64_t dst) {
    unsigned *p = reinterpret_cast<unsigned *>(dst);
#pragma unroll
    for (int i = 0; i < 4; ++i) atomicAdd(p + i, 1u);
}
template <int CNT, typename T>
__device__ __forceinline__ void count_line(T *dst) {
    static_assert(sizeof(T) == 4, "write counts are taken on the FP32 table layout");
    unsigned *p = reinterpret_cast<unsigned *>(dst);
#pragma unroll
    for (int i = 0; i < CNT; ++i) atomicAdd(p + i, 1u);
}

// WALK_REDUCE / WALK_REDUCE_TOP: nothing is written to the table; every lane folds the
// BIC values of its child into a running minimum (with its parent set), a running
// sum of exp(min - BIC) and, for WALK_REDUCE_TOP, the GS_REDUCE_TOPK smallest values
// (with their parent sets), and writes them per (child, segment) at the end.
enum WalkMode { WALK_STORE = 0, WALK_COUNT = 1, WALK_REDUCE = 2, WALK_REDUCE_TOP = 3 };
constexpr float REDUCE_SKIP = 30.0f;  // natural-log units

constexpr int WALK_WAVES = 4;  // waves per workgroup
#ifndef WALK_MIN_WAVES
#define WALK_MIN_WAVES 5
#endif

// The walk of one wave (wave index wid of its dataset's packed wave table).
template <typename T, int KS, bool BIC, int MODE>
__device__ __forceinline__ void walk_body(const T *__restrict__ anchor, const T *__restrict__ tail,
                                          const uint32_t *__restrict__ prog,
                                          const int32_t *__restrict__ lane_seg,
                                          const int8_t *__restrict__ lane_loc,
                                          const int *__restrict__ status,
                                          const ColStats *__restrict__ stats, T *__restrict__ out,
                                          const WalkArgs &a, int64_t wid, T (*L)[64],
                                          float4 *__restrict__ Sg, uint64_t *__restrict__ Dg) {
    constexpr int N = InnerProgram<KS>::N;
    constexpr int NS = 1 << KS;
    const int lane64 = threadIdx.x & 63;
    // this lane's segment and its column slot l inside it
    const int32_t segv = wid < a.nwaves ? lane_seg[wid * 64 + lane64] : -1;
    const bool seg_ok = segv >= 0;
    const int lane = seg_ok ? int(lane_loc[wid * 64 + lane64]) : 63;
    const int m = a.m, k = a.k, q = a.q, nout = m - k;
    const int bbase = (lane64 - (seg_ok ? lane : 0)) * 4;  // ds_bpermute address of slot 0
    // lanes holding inner slot c of their segment (the pivots of the inner walk)
    uint64_t slot_mask[KS];
#pragma unroll
    for (int c = 0; c < KS; ++c) slot_mask[c] = __builtin_amdgcn_ballot_w64(seg_ok && lane == c);

    // slot -> variable label and class: 1 inner, 2 middle, 3 back, 0 unused
    const uint64_t scode = seg_ok ? uint64_t(segv) : 0;
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
    if (!seg_ok) cls = 0;
    const uint64_t Fbits = scode << k;
    const int nF = __popcll((unsigned long long)scode);

    // anchor -> working precision (BIC: rows scaled by 1/sqrt(n))
    const T rs = T(a.row_scale);
    const T *an = anchor + int64_t(seg_ok ? segv : 0) * k * 32 + (seg_ok ? lane : 0);
    T I[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) I[i] = seg_ok ? an[(q + i) * 32] * rs : T(0);
    for (int p = 0; p < q; ++p) L[p][lane64] = seg_ok ? an[p * 32] * rs : T(0);
    const T tl = seg_ok ? tail[int64_t(segv) * 32 + lane] * rs * rs : T(0);
    const T nlog = T(a.nlog), lnn = T(a.lnn);
    // the child's equilibration exponent: BIC offset, RSS factor 2^(2 e_c)
    const int ec2 = label >= 0 ? 2 * stats->exp2[label] : 0;
    const T coff = T(a.nln2 * double(ec2));
    // RSS output only: the largest residual and the smallest non-zero one the lane scored.
    // ldexp by the fixed 2^(2 e_c) never decreases, so some scaled value overflows or a
    // non-zero one underflows exactly when these two do (tested once, after the walk).
    T rss_hi = T(0), rss_lo = T(INFINITY);
    // reduce modes: running minimum, its parent set, sum of exp(min - BIC), top values
    float rmin = __builtin_inff(), rsum = 0.0f;
    uint32_t rmask = 0;
    float tv[GS_REDUCE_TOPK];
    uint32_t tm[GS_REDUCE_TOPK];
#pragma unroll
    for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
        tv[j] = __builtin_inff();
        tm[j] = 0xffffffffu;
    }

    // FP32, inner block 5, table written: the lines of a sub-walk wait in the LDS stage and
    // leave during the next sub-walk, one 16-byte store instruction (8 whole lines) every
    // three inner steps.  Each stage read completes behind the next step's broadcasts, and
    // only one chunk is held in registers at a time (not all eight at the sub-walk's end).
    constexpr bool kStaged =
        std::is_same_v<T, float> && KS == 5 && (MODE == WALK_STORE || MODE == WALK_COUNT);
    static_assert(!kStaged || InnerProgram<KS>::N >= 3 * STAGE_CHUNKS,
                  "every chunk must leave within the next sub-walk's inner steps");
    const int ch = lane64 & 7;
    uint64_t pd = 0;
    float4 pv = make_float4(0.f, 0.f, 0.f, 0.f);
    auto stage_read = [&](int ci, uint64_t &d, float4 &v) {
        const int ow = 8 * ci + (lane64 >> 3);
        d = Dg[ow];
        v = Sg[ch * STAGE_LINES + (ow ^ ch)];
    };
    auto stage_store = [&](uint64_t d, const float4 &v) {
        if (ch < int(d & 15u)) {
            const uint64_t dst = (d & ~uint64_t(15)) + uint64_t(ch) * 16;
            if constexpr (MODE == WALK_COUNT) count16(dst);
            else global_store16(dst, v);
        }
    };
    if constexpr (kStaged) {
        Dg[lane64] = 0;  // nothing staged before the first sub-walk
        wave_lds_sync();
    }

    int z = q;
    // One sub-walk: the transition into it, the inner walk, the table writes.  FWD is
    // the direction of the inner walk (forward on even t), which fixes the inner
    // block's ordering at compile time.
    auto sub_walk = [&](auto gc, auto dirc, uint32_t w0, uint32_t w1) {
        constexpr bool G = decltype(gc)::value;
        constexpr bool FWD = decltype(dirc)::value;
        constexpr auto &ord = FWD ? kInner<KS>.order_f : kInner<KS>.order_r;
        if (w1 & SubWord::kHasTransition) {
            if (w1 & SubWord::kHasMid) {
                // swap of two middle variables on the same side of the inner block
                const int j = int((w1 >> 2) & 31), piv = int((w1 >> 8) & 31);
                const int addr = bbase + piv * 4;
                const T x = L[j][lane64], y = L[j + 1][lane64];
                T c, s;
                givens_cs<G>(bcast(x, addr), bcast(y, addr), c, s);
                L[j][lane64] = c * x + s * y;
                L[j + 1][lane64] = lane == piv ? T(0) : s * x - c * y;
            }
            const int v = int((w1 >> 16) & 31);
            if (w1 & SubWord::kCrossLeft) {
                // middle variable v (first behind the inner block) moves to its front
                T carry = L[z][lane64];
                const int addr = bbase + v * 4;
                static_for<0, KS>([&](auto ic) {
                    constexpr int i = KS - 1 - decltype(ic)::value;
                    T c, s;
                    givens_cs<G>(bcast(I[i], addr), bcast(carry, addr), c, s);
                    const T top = c * I[i] + s * carry;
                    const T bot = s * I[i] - c * carry;
                    I[i] = lane == v ? T(0) : bot;
                    carry = top;
                });
                L[z][lane64] = carry;
                ++z;
            } else {
                // the last front middle variable moves behind the inner block
                T carry = L[z - 1][lane64];
                static_for<0, KS>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int piv = ord[i];
                    const int addr = bbase + piv * 4;
                    T c, s;
                    givens_cs<G>(bcast(carry, addr), bcast(I[i], addr), c, s);
                    const T top = c * carry + s * I[i];
                    carry = select_lanes(slot_mask[piv], T(0), s * carry - c * I[i]);
                    I[i] = top;
                });
                L[z - 1][lane64] = carry;
                --z;
            }
        }

        const uint32_t omask = w0 & 0xFFFFu;
        // suffix sums below the inner block: middle rows behind it and the back rows
        T base = tl;
        for (int p = q - 1; p >= z; --p) {
            const T r = L[p][lane64];
            base = r * r + base;
        }
        T sfx[KS + 1];
        sfx[KS] = base;
#pragma unroll
        for (int i = KS - 1; i >= 0; --i) sfx[i] = I[i] * I[i] + sfx[i + 1];
        T cst[KS + 1];
        const int cnt0 = nF + __popc(omask) + 2;
#pragma unroll
        for (int u = 0; u <= KS; ++u) cst[u] = fma(T(cnt0 + u), lnn, coff);

        T o[NS];
        auto score = [&](T rss, int u) -> T {
            if constexpr (BIC) {
                return Arith<T>::score(rss, nlog, cst[u]);
            } else {
                rss_hi = fmax(rss_hi, rss);
                rss_lo = fmin(rss_lo, rss > T(0) ? rss : T(INFINITY));
                return Arith<T>::ldexp(rss, ec2);
            }
        };
        static_for<0, KS + 1>([&](auto pc) {
            constexpr int pl = decltype(pc)::value;
            constexpr int U = FWD ? kInner<KS>.init_f[pl] : kInner<KS>.init_r[pl];
            o[U] = score(sfx[pl], popcount_c(U));
        });
        static_for<0, N>([&](auto sc) {
            constexpr int st = decltype(sc)::value;
            constexpr int J = FWD ? kInner<KS>.j_f[st] : kInner<KS>.j_r[st];
            constexpr int PV = FWD ? kInner<KS>.piv_f[st] : kInner<KS>.piv_r[st];
            constexpr int U = FWD ? kInner<KS>.mask_f[st] : kInner<KS>.mask_r[st];
            const int addr = bbase + PV * 4;
            T c, s;
            givens_cs<G>(bcast(I[J], addr), bcast(I[J + 1], addr), c, s);
            const T x = I[J], y = I[J + 1];
            I[J] = c * x + s * y;
            const T ny = select_lanes(slot_mask[PV], T(0), s * x - c * y);
            I[J + 1] = ny;
            sfx[J + 1] = ny * ny + sfx[J + 2];
            o[U] = score(sfx[J + 1], popcount_c(U));
            if constexpr (kStaged) {
                // chunk i of the previous sub-walk's lines: read from the stage after
                // step 3i + 1, stored after step 3i + 2 (the read has completed by then)
                constexpr int ci = st / 3;
                if constexpr (ci < STAGE_CHUNKS && st % 3 == 1) stage_read(ci, pd, pv);
                if constexpr (ci < STAGE_CHUNKS && st % 3 == 2) stage_store(pd, pv);
            }
        });

        if constexpr (MODE == WALK_REDUCE || MODE == WALK_REDUCE_TOP) {
            // fold this sub-walk's line into the lane's running reduction
            constexpr float L2E = 1.4426950408889634f;
            const uint32_t Shi32 = uint32_t(Fbits | (uint64_t(omask) << KS));
            const bool is_child =
                cls == 1 || cls == 3 || (cls == 2 && !((omask >> (lane - KS)) & 1u));
            const uint32_t own = cls == 1 ? (1u << lane) : 0u;  // inner child: entries without it
            float v[NS];
            float lmin = __builtin_inff();
            static_for<0, NS>([&](auto uc) {
                constexpr int U = decltype(uc)::value;
                v[U] = (is_child && !(U & own)) ? float(o[U]) : __builtin_inff();
                lmin = fminf(v[U], lmin);
            });
            // Lines whose values all lie more than REDUCE_SKIP above the lane's running
            // minimum add less than e^-REDUCE_SKIP each to the sum of exp(min - BIC) (at
            // most 2^18 per lane and segment: below 3e-8 of the sum, which is >= 1); a
            // wave skips the line when no lane has a value within that distance.
            if (__builtin_amdgcn_ballot_w64(lmin < rmin + REDUCE_SKIP) != 0) {
                const float nm = fminf(rmin, lmin);
                if (__builtin_amdgcn_ballot_w64(lmin < rmin) != 0) {
                    int lU = 0;  // the first entry reaching the line minimum
                    static_for<0, NS>([&](auto uc) {
                        constexpr int U = NS - 1 - decltype(uc)::value;
                        lU = v[U] == lmin ? U : lU;
                    });
                    rmask = lmin < rmin ? (Shi32 | uint32_t(lU)) : rmask;
                }
                float ls = 0.0f;
                static_for<0, NS>([&](auto uc) {
                    constexpr int U = decltype(uc)::value;
                    ls += __builtin_amdgcn_exp2f((nm - v[U]) * L2E);
                });
                if (is_child) {
                    rsum = rsum * __builtin_amdgcn_exp2f((nm - rmin) * L2E) + ls;
                    rmin = nm;
                }
            }
            if constexpr (MODE == WALK_REDUCE_TOP) {
                if (__builtin_amdgcn_ballot_w64(lmin < tv[GS_REDUCE_TOPK - 1]) != 0) {
                    static_for<0, NS>([&](auto uc) {
                        constexpr int U = decltype(uc)::value;
                        float cv = v[U];
                        if (cv < tv[GS_REDUCE_TOPK - 1]) {
                            uint32_t cm = Shi32 | uint32_t(U);
                            static_for<0, GS_REDUCE_TOPK>([&](auto jc) {
                                constexpr int j = decltype(jc)::value;
                                const bool sw = cv < tv[j];
                                const float ov = tv[j];
                                const uint32_t om = tm[j];
                                tv[j] = sw ? cv : ov;
                                tm[j] = sw ? cm : om;
                                cv = sw ? ov : cv;
                                cm = sw ? om : cm;
                            });
                        }
                    });
                }
            }
            return;
        }

        // write this sub-walk's table lines
        const uint64_t Shi = Fbits | (uint64_t(omask) << KS);
        const int lb = label < 0 ? 0 : label;
        const int64_t cbase = int64_t(lb) << (m - 1);
        const bool child = cls == 3 || (cls == 2 && !((omask >> (lane - KS)) & 1u));
        const uint64_t low = Shi & ((uint64_t(1) << lb) - 1);
        const uint64_t high = (Shi >> (lb + 1)) << lb;
        constexpr int NH = NS / 2;
        // inner child c (slot c) writes the entries without its own bit
        // (one select per distinct candidate: the slots whose entries coincide share
        // it, and the most common entry needs none)
        auto inner_entry = [&](auto ic) -> T {
            constexpr int i = decltype(ic)::value;
            constexpr int B = common_expansion(i, KS);
            T val = o[B];
            static_for<0, KS>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                constexpr int e = expand_bit(i, c);
                if constexpr (e != B && first_expansion(i, c)) {
                    uint64_t msk = 0;
                    static_for<c, KS>([&](auto dc) {
                        constexpr int d = decltype(dc)::value;
                        if constexpr (expand_bit(i, d) == e) msk |= slot_mask[d];
                    });
                    val = select_lanes(msk, o[e], val);
                }
            });
            return val;
        };
        if constexpr (std::is_same_v<T, float> && KS == 5) {
            wave_lds_sync();  // the previous sub-walk's stage reads are done
            // One line per lane: its own entries, overridden on inner children's lanes
            // (slot c) by the entries without bit c; those lanes store 4 chunks only.
            auto merged_entry = [&](auto ic) -> T {
                constexpr int i = decltype(ic)::value;
                T val = o[i];
                static_for<0, KS>([&](auto cc) {
                    constexpr int c = decltype(cc)::value;
                    constexpr int e = expand_bit(i, c);
                    if constexpr (e != i && first_expansion(i, c)) {
                        uint64_t msk = 0;
                        static_for<c, KS>([&](auto dc) {
                            constexpr int d = decltype(dc)::value;
                            if constexpr (expand_bit(i, d) == e) msk |= slot_mask[d];
                        });
                        val = select_lanes(msk, o[e], val);
                    }
                });
                return val;
            };
            static_for<0, NS / 4>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                if constexpr (c < NH / 4)
                    Sg[c * STAGE_LINES + (lane64 ^ c)] =
                        make_float4(merged_entry(std::integral_constant<int, 4 * c>{}),
                                    merged_entry(std::integral_constant<int, 4 * c + 1>{}),
                                    merged_entry(std::integral_constant<int, 4 * c + 2>{}),
                                    merged_entry(std::integral_constant<int, 4 * c + 3>{}));
                else
                    Sg[c * STAGE_LINES + (lane64 ^ c)] =
                        make_float4(o[4 * c], o[4 * c + 1], o[4 * c + 2], o[4 * c + 3]);
            });
            const uint64_t inner_dst = reinterpret_cast<uint64_t>(out + cbase + int64_t(Shi >> 1)) | (NH / 4);
            const uint64_t line_dst = reinterpret_cast<uint64_t>(out + cbase + int64_t(low | high)) | (NS / 4);
            Dg[lane64] = cls == 1 ? inner_dst : (child ? line_dst : 0);
            wave_lds_sync();  // staged before any later read of the stage
            // the stores leave during the next sub-walk's inner steps (or after the walk)
        } else {
            if (cls == 1) {
                T h[NH];
                static_for<0, NH>([&](auto ic) { h[decltype(ic)::value] = inner_entry(ic); });
                if constexpr (MODE == WALK_COUNT) count_line<NH>(out + cbase + int64_t(Shi >> 1));
                else store_line<NH>(out + cbase + int64_t(Shi >> 1), h);
            } else if (child) {
                if constexpr (MODE == WALK_COUNT) count_line<NS>(out + cbase + int64_t(low | high));
                else store_line<NS>(out + cbase + int64_t(low | high), o);
            }
        }
    };
    auto run = [&](auto gc) {
        for (int64_t t = 0; t < a.nsub; ++t) {
            const uint32_t w0 = prog[2 * t], w1 = prog[2 * t + 1];
            if ((t & 1) == 0) sub_walk(gc, std::true_type{}, w0, w1);
            else sub_walk(gc, std::false_type{}, w0, w1);
        }
    };
    // The R0 pass has flagged a (near) rank-deficient or very ill-conditioned X: only
    // then can a Givens pivot pair be (near) zero.  The FP64 walk always takes the
    // guarded path.
    if (std::is_same_v<T, double> || (status[0] & GS_FLAG_GUARD)) run(std::true_type{});
    else run(std::false_type{});
    if constexpr (kStaged) {
        wave_lds_sync();  // the last sub-walk's lines are in the stage
        static_for<0, STAGE_CHUNKS>([&](auto cc) {
            constexpr int ci = decltype(cc)::value;
            stage_read(ci, pd, pv);
            stage_store(pd, pv);
        });
    }
    if constexpr (MODE == WALK_REDUCE || MODE == WALK_REDUCE_TOP) {
        if (seg_ok && cls != 0) {
            const int64_t r = int64_t(label) * a.nseg + segv;
            a.red.pmin[r] = rmin;
            a.red.pmask[r] = rmask;
            a.red.psum[r] = rsum;
            if constexpr (MODE == WALK_REDUCE_TOP) {
#pragma unroll
                for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
                    a.red.ptopv[r * GS_REDUCE_TOPK + j] = tv[j];
                    a.red.ptopm[r * GS_REDUCE_TOPK + j] = tm[j];
                }
            }
        }
    }
    if constexpr (!BIC) {
        // an overflow, or an underflow of a non-zero residual (to a subnormal or 0)
        const bool out_of_range = Arith<T>::ldexp(rss_hi, ec2) > Arith<T>::huge() ||
                                  Arith<T>::ldexp(rss_lo, ec2) < Arith<T>::tiny();
        if (__builtin_amdgcn_ballot_w64(out_of_range && seg_ok) != 0 && lane64 == 0)
            atomicOr(const_cast<int *>(status), GS_FLAG_RANGE);
    }
}

template <typename T, int KS, int MODE = WALK_STORE>
__host__ __device__ constexpr size_t walk_stage_bytes() {
    return (std::is_same_v<T, float> && KS == 5 && (MODE == WALK_STORE || MODE == WALK_COUNT))
               ? size_t(STAGE_BYTES)
               : 0;
}
template <typename T, int KS, int MODE = WALK_STORE>
__host__ __device__ constexpr size_t walk_wave_lds(int q) {
    return walk_stage_bytes<T, KS, MODE>() + size_t(q > 0 ? q : 1) * 64 * sizeof(T);
}

template <typename T, int KS, bool BIC, int MINW, int MODE = WALK_STORE>
__global__ __launch_bounds__(64 * WALK_WAVES) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void walk_kernel(const T *__restrict__ anchor, const T *__restrict__ tail,
                 const uint32_t *__restrict__ prog, const int32_t *__restrict__ lane_seg,
                 const int8_t *__restrict__ lane_loc, const int *__restrict__ status,
                 const ColStats *__restrict__ stats, T *__restrict__ out, WalkArgs a) {
    // per wave: the FP32 line stage (inner block 5), then q middle rows of 64 entries
    extern __shared__ float4 lds_walk[];
    const int wave = threadIdx.x >> 6;
    const int64_t wid = int64_t(blockIdx.x) * WALK_WAVES + wave;
    char *base = reinterpret_cast<char *>(lds_walk) + wave * walk_wave_lds<T, KS, MODE>(a.q);
    constexpr size_t stage = walk_stage_bytes<T, KS, MODE>();
    float4 *Sg = reinterpret_cast<float4 *>(base);
    uint64_t *Dg = reinterpret_cast<uint64_t *>(base + STAGE_LINES * STAGE_CHUNKS * 16);
    walk_body<T, KS, BIC, MODE>(anchor, tail, prog, lane_seg, lane_loc, status, stats, out, a, wid,
                          reinterpret_cast<T(*)[64]>(base + stage), Sg, Dg);
}

// Many datasets in one launch: wave gw walks wave wave_local[gw] of dataset
// wave_item[gw] (the host orders the waves longest walk first).
template <typename T, int KS, bool BIC, int MINW>
__global__ __launch_bounds__(64 * WALK_WAVES) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void walk_batched_kernel(const BatchItem *__restrict__ items, const int32_t *__restrict__ wave_item,
                         const int32_t *__restrict__ wave_local, int64_t total_waves, int qmax) {
    extern __shared__ float4 lds_walk[];
    const int wave = threadIdx.x >> 6;
    const int64_t gw = int64_t(blockIdx.x) * WALK_WAVES + wave;
    if (gw >= total_waves) return;
    char *base = reinterpret_cast<char *>(lds_walk) + wave * walk_wave_lds<T, KS>(qmax);
    constexpr size_t stage = walk_stage_bytes<T, KS>();
    float4 *Sg = reinterpret_cast<float4 *>(base);
    uint64_t *Dg = reinterpret_cast<uint64_t *>(base + STAGE_LINES * STAGE_CHUNKS * 16);
    const BatchItem &d = items[wave_item[gw]];
    WalkArgs a;
    a.m = d.m;
    a.k = d.k;
    a.q = d.q;
    a.nseg = d.nseg;
    a.nsub = d.nsub;
    a.nwaves = d.nwaves;
    a.row_scale = d.row_scale;
    a.nlog = d.nlog;
    a.lnn = d.lnn;
    a.nln2 = d.nln2;
    walk_body<T, KS, BIC, WALK_STORE>(static_cast<const T *>(d.anchor),
                                      static_cast<const T *>(d.tail), d.prog,
                          d.lane_seg, d.lane_loc, d.status, d.stats, static_cast<T *>(d.out), a,
                          wave_local[gw], reinterpret_cast<T(*)[64]>(base + stage), Sg, Dg);
}

// Register budget: the FP32 kernel with inner block 5 is held to 128 VGPRs (4 waves
// per SIMD; its 8 KB line stage allows no more), smaller inner blocks to 96 VGPRs
// (5 waves per SIMD); the others take what they need.
template <typename T, int KS>
constexpr int kMinWaves = !std::is_same_v<T, float> ? 1 : (KS == 5 ? 4 : (KS < 5 ? WALK_MIN_WAVES : 1));
// the top-k reduction keeps 16 more values per lane and has no line stage: 168 VGPRs
// with inner block 5, 128 with smaller ones
template <typename T, int KS, int MODE>
constexpr int kMinWavesMode =
    MODE == WALK_REDUCE_TOP ? (KS == 5 ? 3 : (KS < 5 ? 4 : 1)) : kMinWaves<T, KS>;
// the FP32 RSS table with inner block 5 gets 168 VGPRs too: held to 128 it spilled to
// scratch and took three times as long as the BIC walk
template <typename T, int KS, bool BIC, int MODE>
constexpr int kMinW = (!BIC && std::is_same_v<T, float> && KS == 5) ? 3 : kMinWavesMode<T, KS, MODE>;

template <typename T, bool BIC, int MODE = WALK_STORE>
static hipError_t launch_walk_t(const gs_plan_s *p, const WalkTables &t, const T *anchor,
                                const T *tail, T *out, int64_t n, hipStream_t s,
                                const ReducePartials *red = nullptr) {
    WalkArgs a;
    a.red = red ? *red : ReducePartials{};
    a.m = p->m;
    a.k = p->k;
    a.q = p->q;
    a.nseg = p->nseg;
    a.nsub = p->nsub;
    a.nwaves = p->nwaves;
    const double dn = double(n);
    a.row_scale = BIC ? 1.0 / std::sqrt(dn) : 1.0;
    a.nlog = std::is_same_v<T, float> ? dn * 0.6931471805599453 : dn;
    a.lnn = std::log(dn);
    a.nln2 = dn * 0.6931471805599453;
    const dim3 grid(unsigned((p->nwaves + WALK_WAVES - 1) / WALK_WAVES));
    const dim3 block(64 * WALK_WAVES);
    const size_t lds = WALK_WAVES * (p->ks == 5 ? walk_wave_lds<T, 5, MODE>(p->q)
                                                : walk_wave_lds<T, 1, MODE>(p->q));
    switch (p->ks) {
#define GS_WALK_CASE(KSV)                                                                   \
    case KSV:                                                                               \
        hipLaunchKernelGGL((walk_kernel<T, KSV, BIC, kMinW<T, KSV, BIC, MODE>, MODE>), grid,  \
                           block, lds,                                                         \
                           s,                                                                  \
                           anchor, tail,                                                    \
                           t.prog, t.lane_seg, t.lane_loc, t.status, t.stats, out, a);      \
        break;
        GS_WALK_CASE(1)
        GS_WALK_CASE(2)
        GS_WALK_CASE(3)
        GS_WALK_CASE(4)
        GS_WALK_CASE(5)
        GS_WALK_CASE(6)
#undef GS_WALK_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_walk_batched_f32(const BatchItem *items, const int32_t *wave_item,
                                   const int32_t *wave_local, int64_t total_waves, int qmax,
                                   bool bic, hipStream_t s) {
    const size_t lds = WALK_WAVES * walk_wave_lds<float, 5>(qmax);
    const dim3 grid(unsigned((total_waves + WALK_WAVES - 1) / WALK_WAVES)), block(64 * WALK_WAVES);
    if (bic)
        hipLaunchKernelGGL((walk_batched_kernel<float, 5, true, kMinWaves<float, 5>>), grid, block, lds,
                           s, items, wave_item, wave_local, total_waves, qmax);
    else
        hipLaunchKernelGGL((walk_batched_kernel<float, 5, false, kMinW<float, 5, false, WALK_STORE>>), grid, block,
                           lds, s, items, wave_item, wave_local, total_waves, qmax);
    return hipGetLastError();
}

static WalkTables plan_tables(const gs_plan_s *p) {
    return WalkTables{p->d_prog, p->d_lane_seg, p->d_lane_loc, p->d_status, p->d_stats};
}

hipError_t launch_walk_f32_tables(const gs_plan_s *p, const WalkTables &t, const float *anchor,
                                  const float *tail, float *out, int64_t n, bool bic,
                                  hipStream_t s) {
    return bic ? launch_walk_t<float, true>(p, t, anchor, tail, out, n, s)
               : launch_walk_t<float, false>(p, t, anchor, tail, out, n, s);
}

hipError_t launch_walk_f32(const gs_plan_s *p, const float *anchor, const float *tail, float *out,
                           int64_t n, bool bic, hipStream_t s) {
    return launch_walk_f32_tables(p, plan_tables(p), anchor, tail, out, n, bic, s);
}

hipError_t launch_walk_count(const gs_plan_s *p, const float *anchor, const float *tail,
                             uint32_t *counts, int64_t n, hipStream_t s) {
    return launch_walk_t<float, true, WALK_COUNT>(p, plan_tables(p), anchor, tail,
                                                  reinterpret_cast<float *>(counts), n, s);
}

hipError_t launch_walk_reduce(const gs_plan_s *p, const float *anchor, const float *tail,
                              const ReducePartials &red, bool top, int64_t n, hipStream_t s) {
    return top ? launch_walk_t<float, true, WALK_REDUCE_TOP>(p, plan_tables(p), anchor, tail,
                                                             nullptr, n, s, &red)
               : launch_walk_t<float, true, WALK_REDUCE>(p, plan_tables(p), anchor, tail, nullptr,
                                                         n, s, &red);
}

hipError_t launch_walk_f64(const gs_plan_s *p, const double *anchor, const double *tail,
                           double *out, int64_t n, bool bic, hipStream_t s) {
    return bic ? launch_walk_t<double, true>(p, plan_tables(p), anchor, tail, out, n, s)
               : launch_walk_t<double, false>(p, plan_tables(p), anchor, tail, out, n, s);
}

}  // namespace gs
