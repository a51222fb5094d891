// Per-child merge of the fused reduction (gs_score_reduce).
//
// Score-based learning consumes the local scores of all families (Sec. 1): per child
// the best parent set, a short list of the best ones, or a soft-min over all of them.
// The walk in a reduce mode folds its BIC values per (child, segment) instead of
// writing the m 2^(m-1) table; here fixed slices of each child's segment partials
// are merged by up to GS_REDUCE_SPLIT workgroups per child and those results by one
// wave per child, always in the same order (the result is reproducible bit for bit):
//   best[c]      = min over S of BIC(c, S), best_mask[c] a parent set reaching it (on
//                  equal values the smaller mask);
//   lse[c]       = ln sum_S exp(-BIC(c, S)), accumulated relative to the running minimum
//                  in double;
//   top_v, top_m = the top_k smallest BIC values of the child, ascending, with their
//                  parent sets.
// A walked variable (label < k) is a child in every segment; a variable k + b of the
// outer block only in the segments that put it behind the walked block (bit b = 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gs_internal.hpp"

namespace gs {

constexpr int RED_THREADS = 256;

struct MinSum {
    double mn;   // minimum BIC so far
    double sum;  // sum of exp(mn - BIC)
    uint32_t mask;
};

__device__ __forceinline__ void merge(MinSum &a, double mn, double sum, uint32_t mask) {
    if (!(sum > 0.0)) return;  // nothing folded (or an empty segment)
    const double m2 = fmin(a.mn, mn);
    const double s2 = a.sum * exp(m2 - a.mn) + sum * exp(m2 - mn);
    if (mn < a.mn || (mn == a.mn && mask < a.mask)) a.mask = mask;
    a.mn = m2;
    a.sum = s2;
}

__device__ __forceinline__ void top_insert(float (&tv)[GS_REDUCE_TOPK],
                                           uint32_t (&tm)[GS_REDUCE_TOPK], float v, uint32_t mk) {
    if (!(v < __builtin_inff())) return;  // an unused slot
    if (!(v < tv[GS_REDUCE_TOPK - 1] ||
          (v == tv[GS_REDUCE_TOPK - 1] && mk < tm[GS_REDUCE_TOPK - 1])))
        return;
#pragma unroll
    for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
        const bool sw = v < tv[j] || (v == tv[j] && mk < tm[j]);
        const float ov = tv[j];
        const uint32_t om = tm[j];
        tv[j] = sw ? v : ov;
        tm[j] = sw ? mk : om;
        v = sw ? ov : v;
        mk = sw ? om : mk;
    }
}

// Stage 1: workgroup (part, c) reduces the segments part * 256 + t + j * split * 256 of
// child c (thread t, j = 0, 1, ...), first per thread in that order, then by a fixed
// tree over the threads, into stage[c * GS_REDUCE_SPLIT + part].
template <bool TOP>
__global__ __launch_bounds__(RED_THREADS) void reduce_slices_kernel(ReducePartials red, int k,
                                                                    int64_t nseg, int split) {
    __shared__ double s_mn[RED_THREADS], s_sum[RED_THREADS];
    __shared__ uint32_t s_mask[RED_THREADS];
    __shared__ float s_tv[TOP ? RED_THREADS : 1][GS_REDUCE_TOPK];
    __shared__ uint32_t s_tm[TOP ? RED_THREADS : 1][GS_REDUCE_TOPK];
    const int part = blockIdx.x;
    const int c = blockIdx.y;
    const int t = threadIdx.x;
    MinSum acc{__builtin_inf(), 0.0, 0xffffffffu};
    float tv[GS_REDUCE_TOPK];
    uint32_t tm[GS_REDUCE_TOPK];
#pragma unroll
    for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
        tv[j] = __builtin_inff();
        tm[j] = 0xffffffffu;
    }
    const bool walked = c < k;
    const int64_t stride = int64_t(split) * RED_THREADS;
    for (int64_t sg = int64_t(part) * RED_THREADS + t; sg < nseg; sg += stride) {
        if (!walked && ((sg >> (c - k)) & 1)) continue;  // c is a front variable there
        const int64_t r = int64_t(c) * nseg + sg;
        merge(acc, double(red.pmin[r]), double(red.psum[r]), red.pmask[r]);
        if constexpr (TOP) {
            // a segment's list is ascending in value: past a value above the current
            // 8th best no later one can enter
#pragma unroll
            for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
                const float v = red.ptopv[r * GS_REDUCE_TOPK + j];
                if (v > tv[GS_REDUCE_TOPK - 1]) break;
                top_insert(tv, tm, v, red.ptopm[r * GS_REDUCE_TOPK + j]);
            }
        }
    }
    s_mn[t] = acc.mn;
    s_sum[t] = acc.sum;
    s_mask[t] = acc.mask;
    if constexpr (TOP) {
#pragma unroll
        for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
            s_tv[t][j] = tv[j];
            s_tm[t][j] = tm[j];
        }
    }
    __syncthreads();
    for (int half = RED_THREADS / 2; half >= 1; half >>= 1) {
        if (t < half) {
            merge(acc, s_mn[t + half], s_sum[t + half], s_mask[t + half]);
            s_mn[t] = acc.mn;
            s_sum[t] = acc.sum;
            s_mask[t] = acc.mask;
            if constexpr (TOP) {
#pragma unroll
                for (int j = 0; j < GS_REDUCE_TOPK; ++j)
                    top_insert(tv, tm, s_tv[t + half][j], s_tm[t + half][j]);
#pragma unroll
                for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
                    s_tv[t][j] = tv[j];
                    s_tm[t][j] = tm[j];
                }
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        ReduceStage &o = red.stage[c * GS_REDUCE_SPLIT + part];
        o.mn = acc.mn;
        o.sum = acc.sum;
        o.mask = acc.mask;
#pragma unroll
        for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
            o.tv[j] = tv[j];
            o.tm[j] = tm[j];
        }
    }
}

// Stage 2: one wave per child merges its split stage records by a fixed tree.
template <bool TOP>
__global__ __launch_bounds__(64) void reduce_children_kernel(
    ReducePartials red, int split, float *__restrict__ best, uint32_t *__restrict__ best_mask,
    double *__restrict__ lse, float *__restrict__ top_v, uint32_t *__restrict__ top_m,
    int top_k) {
    __shared__ ReduceStage s_st[GS_REDUCE_SPLIT];
    const int c = blockIdx.x;
    const int t = threadIdx.x;
    MinSum acc{__builtin_inf(), 0.0, 0xffffffffu};
    float tv[GS_REDUCE_TOPK];
    uint32_t tm[GS_REDUCE_TOPK];
#pragma unroll
    for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
        tv[j] = __builtin_inff();
        tm[j] = 0xffffffffu;
    }
    if (t < split) {
        const ReduceStage &in = red.stage[c * GS_REDUCE_SPLIT + t];
        merge(acc, in.mn, in.sum, in.mask);
        if constexpr (TOP) {
#pragma unroll
            for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
                tv[j] = in.tv[j];
                tm[j] = in.tm[j];
            }
        }
    }
    if (t < GS_REDUCE_SPLIT) {
        s_st[t].mn = acc.mn;
        s_st[t].sum = acc.sum;
        s_st[t].mask = acc.mask;
#pragma unroll
        for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
            s_st[t].tv[j] = tv[j];
            s_st[t].tm[j] = tm[j];
        }
    }
    __syncthreads();
    for (int half = GS_REDUCE_SPLIT / 2; half >= 1; half >>= 1) {
        if (t < half) {
            const ReduceStage &o = s_st[t + half];
            merge(acc, o.mn, o.sum, o.mask);
            if constexpr (TOP) {
#pragma unroll
                for (int j = 0; j < GS_REDUCE_TOPK; ++j) top_insert(tv, tm, o.tv[j], o.tm[j]);
            }
        }
        __syncthreads();
        if (t < half) {
            s_st[t].mn = acc.mn;
            s_st[t].sum = acc.sum;
            s_st[t].mask = acc.mask;
#pragma unroll
            for (int j = 0; j < GS_REDUCE_TOPK; ++j) {
                s_st[t].tv[j] = tv[j];
                s_st[t].tm[j] = tm[j];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        best[c] = float(acc.mn);
        best_mask[c] = acc.mask;
        lse[c] = -acc.mn + log(acc.sum);
        if constexpr (TOP) {
            for (int j = 0; j < top_k; ++j) {
                top_v[c * top_k + j] = tv[j];
                top_m[c * top_k + j] = tm[j];
            }
        }
    }
}

hipError_t launch_reduce_children(const gs_plan_s *p, const ReducePartials &red, bool top,
                                  float *best, uint32_t *best_mask, double *lse, float *top_v,
                                  uint32_t *top_m, int top_k, hipStream_t s) {
    const int split =
        int(std::min<int64_t>(GS_REDUCE_SPLIT, (p->nseg + RED_THREADS - 1) / RED_THREADS));
    const dim3 g1(unsigned(split), unsigned(p->m));
    if (top) {
        hipLaunchKernelGGL(reduce_slices_kernel<true>, g1, dim3(RED_THREADS), 0, s, red, p->k,
                           p->nseg, split);
        hipLaunchKernelGGL(reduce_children_kernel<true>, dim3(unsigned(p->m)), dim3(64), 0, s, red,
                           split, best, best_mask, lse, top_v, top_m, top_k);
    } else {
        hipLaunchKernelGGL(reduce_slices_kernel<false>, g1, dim3(RED_THREADS), 0, s, red, p->k,
                           p->nseg, split);
        hipLaunchKernelGGL(reduce_children_kernel<false>, dim3(unsigned(p->m)), dim3(64), 0, s,
                           red, split, best, best_mask, lse, top_v, top_m, top_k);
    }
    return hipGetLastError();
}

}  // namespace gs
