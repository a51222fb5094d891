// C-ABI entry points of libgivscore that touch the device: argument checks,
// workspace management, the launch sequence R0 -> anchors -> walk, the status
// word and the per-stage timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <vector>
#include <string>

#include "gs_internal.hpp"

using namespace gs;

namespace {

void free_device(gs_plan_s *p) {
    if (p->done) (void)hipEventDestroy(p->done);
    for (auto &ev : p->events)
        for (auto e : ev) (void)hipEventDestroy(e);
    p->events.clear();
    (void)hipFree(p->d_prog);
    (void)hipFree(p->d_lane_seg);
    (void)hipFree(p->d_lane_loc);
    p->d_lane_seg = nullptr;
    p->d_lane_loc = nullptr;
    (void)hipFree(p->d_r0);
    (void)hipFree(p->d_qr_a);
    (void)hipFree(p->d_qr_b);
    (void)hipFree(p->d_anchor);
    (void)hipFree(p->d_tail);
    (void)hipFree(p->d_status);
    (void)hipFree(p->d_stats);
    p->d_stats = nullptr;
    (void)hipFree(p->d_anchorbar);
    (void)hipFree(p->d_tailbar);
    (void)hipFree(p->d_vout);
    (void)hipFree(p->d_partial);
    (void)hipFree(p->d_B);
    (void)hipFree(p->d_K);
    (void)hipFree(p->d_anchor_end);
    p->d_anchor_end = nullptr;
    (void)hipFree(p->d_ups);
    p->d_ups = nullptr;
    p->beta_k = 0;
    (void)hipFree(p->red.pmin);
    (void)hipFree(p->red.pmask);
    (void)hipFree(p->red.psum);
    (void)hipFree(p->red.ptopv);
    (void)hipFree(p->red.ptopm);
    (void)hipFree(p->red.stage);
    p->red = ReducePartials{};
    p->d_anchorbar = p->d_tailbar = p->d_vout = p->d_partial = p->d_B = p->d_K = nullptr;
    p->d_prog = nullptr;
    p->d_r0 = p->d_qr_a = p->d_qr_b = nullptr;
    p->d_anchor = p->d_tail = nullptr;
    p->d_status = nullptr;
    p->done = nullptr;
    p->qr_cap = 0;
    p->device = -1;
}

// Device bytes a plan holds after a call with n rows (the adjoint's extra buffers
// with backward != 0).
int64_t workspace_bytes(const gs_plan_s *p, int64_t n, bool backward) {
    const int64_t m2 = int64_t(p->m) * p->m;
    int64_t b = int64_t(p->prog.size()) * 4 + int64_t(p->lane_seg.size()) * 4 +
                int64_t(p->lane_loc.size()) + m2 * 8 + p->nseg * p->k * 32 * 8 + p->nseg * 32 * 8 +
                int64_t(sizeof(int)) * 4 + int64_t(sizeof(ColStats)) +
                2 * qr_workspace_elems(n, p->m) * 8;
    if (backward)
        b += p->nseg * p->k * 32 * 8 * (p->k >= ADJ_END_MIN_K ? 2 : 1) + p->nseg * 32 * 8 +
             p->nseg * m2 * 8 + adjoint_partial_chunks(p->nseg) * m2 * 8 + 2 * m2 * 8;
    return b;
}

// A cap on the workspace from the environment (GS_WORKSPACE_LIMIT, bytes), checked
// before any device call: a host-forced GS_ENOMEM for callers and tests.
int check_workspace_cap(const gs_plan_s *p, int64_t n, bool backward) {
    const char *env = std::getenv("GS_WORKSPACE_LIMIT");
    if (!env || !*env) return GS_OK;
    char *end = nullptr;
    const long long cap = std::strtoll(env, &end, 10);
    if (end == env || cap < 0) return fail(GS_EINVAL, "GS_WORKSPACE_LIMIT is not a byte count");
    const int64_t need = workspace_bytes(p, n, backward);
    if (need > cap)
        return fail(GS_ENOMEM, "workspace of " + std::to_string(need) +
                                   " bytes exceeds GS_WORKSPACE_LIMIT=" + std::to_string(cap));
    return GS_OK;
}

int ensure_workspace(gs_plan_s *p, int64_t n) {
    int st = check_workspace_cap(p, n, false);
    if (st != GS_OK) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (p->device >= 0 && p->device != dev)
        return fail(GS_EINVAL, "plan was first used on another device");
    if (p->device < 0) {
        p->device = dev;
        const size_t prog_b = p->prog.size() * sizeof(uint32_t);
        const size_t r0_b = size_t(p->m) * p->m * sizeof(double);
        const size_t an_b = size_t(p->nseg) * p->k * 32 * sizeof(double);
        const size_t tl_b = size_t(p->nseg) * 32 * sizeof(double);
        const size_t ls_b = p->lane_seg.size() * sizeof(int32_t);
        const size_t ll_b = p->lane_loc.size() * sizeof(int8_t);
        if ((e = hipMalloc(&p->d_prog, prog_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_lane_seg, ls_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_lane_loc, ll_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_r0, r0_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_anchor, an_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_tail, tl_b)) != hipSuccess ||
            (e = hipMalloc(&p->d_status, sizeof(int) * 4)) != hipSuccess ||
            (e = hipMalloc(&p->d_stats, sizeof(ColStats))) != hipSuccess) {
            free_device(p);
            return fail(GS_ENOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
        }
        if ((e = hipMemcpy(p->d_prog, p->prog.data(), prog_b, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(p->d_lane_seg, p->lane_seg.data(), ls_b, hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemcpy(p->d_lane_loc, p->lane_loc.data(), ll_b, hipMemcpyHostToDevice)) !=
                hipSuccess ||
            (e = hipMemset(p->d_status, 0, sizeof(int) * 4)) != hipSuccess ||
            (e = hipMemset(p->d_stats, 0, sizeof(ColStats))) != hipSuccess ||
            (e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming)) != hipSuccess) {
            free_device(p);
            return hip_fail(e, "workspace initialisation");
        }
    }
    const int64_t need = qr_workspace_elems(n, p->m);
    if (need > p->qr_cap) {
        (void)hipFree(p->d_qr_a);
        (void)hipFree(p->d_qr_b);
        p->d_qr_a = p->d_qr_b = nullptr;
        p->qr_cap = 0;
        if ((e = hipMalloc(&p->d_qr_a, size_t(need) * sizeof(double))) != hipSuccess ||
            (e = hipMalloc(&p->d_qr_b, size_t(need) * sizeof(double))) != hipSuccess) {
            (void)hipFree(p->d_qr_a);
            p->d_qr_a = nullptr;
            return fail(GS_ENOMEM, std::string("QR workspace allocation failed: ") + hipGetErrorString(e));
        }
        p->qr_cap = need;
    }
    return GS_OK;
}

int check_common(gs_plan_s *p, const void *X, int64_t n, int m, int64_t ldx, const void *out,
                 const char *who) {
    const std::string w(who);
    if (!p) return fail(GS_EINVAL, w + ": plan is NULL");
    if (!X || !out) return fail(GS_EINVAL, w + ": NULL data pointer");
    if (m != p->m) return fail(GS_EINVAL, w + ": m differs from the plan's m");
    if (n <= m) return fail(GS_EINVAL, w + ": need n > m samples");
    if (ldx < m) return fail(GS_EINVAL, w + ": ldx < m");
    if (reinterpret_cast<uintptr_t>(out) % 16 != 0)
        return fail(GS_EINVAL, w + ": output must be 16-byte aligned");
    return GS_OK;
}

// Enqueue R0 and the anchors (stored as T); returns GS_OK or an error code.
template <typename T>
int front_half(gs_plan_s *p, const double *X, int64_t n, int m, int64_t ldx, hipStream_t s,
               hipEvent_t *ev) {
    hipError_t e;
    p->front_x = nullptr;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = launch_front_reset(p->d_status, p->d_stats, 1, s)) != hipSuccess)
        return hip_fail(e, "status reset launch");
    if ((e = launch_qr_r0(X, n, m, ldx, p->d_r0, nullptr, p->d_qr_a, p->d_qr_b, p->d_status,
                          p->d_stats, s)) != hipSuccess)
        return hip_fail(e, "R0 QR launch");
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = launch_anchors<T>(p->d_r0, p->d_stats, p->m, p->k, p->ks, p->nseg,
                               static_cast<T *>(p->d_anchor), static_cast<T *>(p->d_tail), s)) !=
        hipSuccess)
        return hip_fail(e, "anchor launch");
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->front_x = X;
    p->front_n = n;
    p->front_ldx = ldx;
    p->front_elem = int(sizeof(T));
    return GS_OK;
}

hipEvent_t *new_event_set(gs_plan_s *p) {
    if (!p->timing) return nullptr;
    std::array<hipEvent_t, 4> ev{};
    for (auto &x : ev)
        if (hipEventCreate(&x) != hipSuccess) return nullptr;
    p->events.push_back(ev);
    return p->events.back().data();
}

template <typename T>
int score_all_impl(gs_plan_s *p, const double *X, int64_t n, int m, int64_t ldx, T *scores,
                   int what, void *stream, const char *who) {
    int st = check_common(p, X, n, m, ldx, scores, who);
    if (st != GS_OK) return st;
    if (what != GS_OUT_BIC && what != GS_OUT_RSS)
        return fail(GS_EINVAL, std::string(who) + ": what must be GS_OUT_BIC or GS_OUT_RSS");
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t *ev = new_event_set(p);
    if ((st = front_half<T>(p, X, n, m, ldx, s, ev)) != GS_OK) return st;
    hipError_t e;
    const T *an = static_cast<const T *>(p->d_anchor), *tl = static_cast<const T *>(p->d_tail);
    if constexpr (std::is_same_v<T, float>)
        e = launch_walk_f32(p, an, tl, scores, n, what == GS_OUT_BIC, s);
    else
        e = launch_walk_f64(p, an, tl, scores, n, what == GS_OUT_BIC, s);
    if (e != hipSuccess) return hip_fail(e, "walk launch");
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->last_stream = s;
    return GS_OK;
}

int ensure_adjoint_workspace(gs_plan_s *p, int64_t n) {
    if (p->d_anchorbar) return GS_OK;
    int st = check_workspace_cap(p, n, true);
    if (st != GS_OK) return st;
    const size_t m2 = size_t(p->m) * p->m;
    const size_t nch = size_t(adjoint_partial_chunks(p->nseg));
    hipError_t e;
    if ((e = hipMalloc(&p->d_anchorbar, size_t(p->nseg) * p->k * 32 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_tailbar, size_t(p->nseg) * 32 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_vout, size_t(p->nseg) * m2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_partial, nch * m2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_B, m2 * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_K, m2 * sizeof(double))) != hipSuccess ||
        (p->k >= ADJ_END_MIN_K &&
         (e = hipMalloc(&p->d_anchor_end, size_t(p->nseg) * p->k * 32 * sizeof(double))) !=
             hipSuccess)) {
        (void)hipFree(p->d_anchorbar);
        (void)hipFree(p->d_tailbar);
        (void)hipFree(p->d_vout);
        (void)hipFree(p->d_partial);
        (void)hipFree(p->d_B);
        (void)hipFree(p->d_K);
        p->d_anchorbar = p->d_tailbar = p->d_vout = p->d_partial = p->d_B = p->d_K = nullptr;
        return fail(GS_ENOMEM, std::string("adjoint workspace allocation failed: ") +
                                   hipGetErrorString(e));
    }
    return GS_OK;
}

template <typename T>
int score_backward_impl(gs_plan_s *p, const double *X, int64_t n, int m, int64_t ldx,
                        const T *dscores, int what, double *dX, int64_t lddx, void *stream,
                        const char *who) {
    int st = check_common(p, X, n, m, ldx, dX, who);
    if (st != GS_OK) return st;
    if (!dscores) return fail(GS_EINVAL, std::string(who) + ": dscores is NULL");
    if (reinterpret_cast<uintptr_t>(dscores) % 16 != 0)
        return fail(GS_EINVAL, std::string(who) + ": dscores must be 16-byte aligned");
    if (lddx < m) return fail(GS_EINVAL, std::string(who) + ": lddx < m");
    if (what != GS_OUT_BIC && what != GS_OUT_RSS)
        return fail(GS_EINVAL, std::string(who) + ": what must be GS_OUT_BIC or GS_OUT_RSS");
    if ((st = check_workspace_cap(p, n, true)) != GS_OK) return st;
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    if ((st = ensure_adjoint_workspace(p, n)) != GS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // R0 and the anchors of the plan's last call on the same data, if allowed and present
    const bool reuse = p->reuse_front && p->front_x == X && p->front_n == n &&
                       p->front_ldx == ldx && p->front_elem == int(sizeof(T));
    if (!reuse && (st = front_half<T>(p, X, n, m, ldx, s, nullptr)) != GS_OK) return st;
    hipError_t e = hipSuccess;
    T *an_end = nullptr;  // long walks start the reverse walk from their end state
    if (p->k >= ADJ_END_MIN_K) {
        an_end = static_cast<T *>(p->d_anchor_end);
        if ((e = launch_anchors_end<T>(p->d_r0, p->d_stats, p->m, p->k, p->ks, p->nseg, p->end,
                                       an_end, s)) != hipSuccess)
            return hip_fail(e, "end-state anchor launch");
    }
    e = launch_walk_adjoint<T>(p, static_cast<const T *>(p->d_anchor),
                                          static_cast<const T *>(p->d_tail), an_end, dscores,
                                          p->d_anchorbar, p->d_tailbar, n, what == GS_OUT_BIC, s);
    if (e != hipSuccess) return hip_fail(e, "walk adjoint launch");
    if ((e = launch_qr_adjoint_chain(p, p->d_r0, p->d_stats, what == GS_OUT_BIC, p->d_anchorbar,
                                     p->d_tailbar, p->d_vout,
                                     p->d_partial, p->d_B, p->d_K, X, n, ldx, dX, lddx, s)) !=
        hipSuccess)
        return hip_fail(e, "QR adjoint launch");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return GS_OK;
}

}  // namespace

extern "C" {

int gs_score_backward(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx,
                      const float *dscores, int what, double *dX, int64_t lddx, void *stream) {
    return score_backward_impl<float>(p, X, n, m, ldx, dscores, what, dX, lddx, stream,
                                      "gs_score_backward");
}

int gs_score_backward_f64(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx,
                          const double *dscores, int what, double *dX, int64_t lddx, void *stream) {
    return score_backward_impl<double>(p, X, n, m, ldx, dscores, what, dX, lddx, stream,
                                       "gs_score_backward_f64");
}

int gs_plan_set_reuse(gs_plan_t *p, int enable) {
    if (!p) return fail(GS_EINVAL, "gs_plan_set_reuse: plan is NULL");
    p->reuse_front = enable != 0;
    return GS_OK;
}


void gs_plan_destroy(gs_plan_t *p) {
    if (!p) return;
    if (p->device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(p->device);
        for (hipEvent_t e : p->slot_join) (void)hipEventSynchronize(e);
        if (p->done) (void)hipEventSynchronize(p->done);
        for (hipEvent_t e : p->slot_join) (void)hipEventDestroy(e);
        for (hipStream_t s : p->slot_streams) (void)hipStreamDestroy(s);
        if (p->fork) (void)hipEventDestroy(p->fork);
        (void)hipFree(p->d_many_status);
        free_device(p);
        (void)hipSetDevice(cur);
    }
    for (gs_plan_s *q : p->slots) gs_plan_destroy(q);
    delete p;
}

int gs_score_all_many(gs_plan_t *p, int count, const double *const *X, int64_t n, int64_t ldx,
                      float *const *scores, int what, int in_flight, void *stream) {
    const char *who = "gs_score_all_many";
    if (!p || !X || !scores) return fail(GS_EINVAL, "gs_score_all_many: NULL argument");
    if (count < 1) return fail(GS_EINVAL, "gs_score_all_many: count must be positive");
    if (in_flight < 1 || in_flight > GS_MANY_MAX_IN_FLIGHT)
        return fail(GS_EINVAL, "gs_score_all_many: in_flight must be in 1..8");
    if (what != GS_OUT_BIC && what != GS_OUT_RSS)
        return fail(GS_EINVAL, "gs_score_all_many: what must be GS_OUT_BIC or GS_OUT_RSS");
    int st;
    for (int i = 0; i < count; ++i)
        if ((st = check_common(p, X[i], n, p->m, ldx, scores[i], who)) != GS_OK) return st;
    in_flight = std::min(in_flight, count);
    while (int(p->slots.size()) < in_flight - 1) {
        gs_plan_t *q = nullptr;
        if ((st = gs_plan_tuned(p->m, p->k, p->ks, &q)) != GS_OK) return st;
        p->slots.push_back(q);
    }
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    hipError_t e;
    if (!p->fork && (e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    while (int(p->slot_streams.size()) < in_flight) {
        hipStream_t t = nullptr;
        hipEvent_t j = nullptr;
        if ((e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreate");
        if ((e = hipEventCreateWithFlags(&j, hipEventDisableTiming)) != hipSuccess) {
            (void)hipStreamDestroy(t);
            return hip_fail(e, "hipEventCreate");
        }
        p->slot_streams.push_back(t);
        p->slot_join.push_back(j);
    }
    if (count > p->many_cap) {
        // the previous call may still write its status words
        for (hipEvent_t j : p->slot_join)
            if ((e = hipEventSynchronize(j)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        (void)hipFree(p->d_many_status);
        p->d_many_status = nullptr;
        p->many_cap = 0;
        if ((e = hipMalloc(&p->d_many_status, size_t(count) * sizeof(int))) != hipSuccess)
            return fail(GS_ENOMEM, std::string("gs_score_all_many: status words: ") +
                                       hipGetErrorString(e));
        p->many_cap = count;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((e = hipEventRecord(p->fork, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    for (int j = 0; j < in_flight; ++j)
        if ((e = hipStreamWaitEvent(p->slot_streams[j], p->fork, 0)) != hipSuccess)
            return hip_fail(e, "hipStreamWaitEvent");
    st = GS_OK;
    for (int i = 0; i < count && st == GS_OK; ++i) {
        const int j = i % in_flight;
        gs_plan_s *q = j == 0 ? p : p->slots[j - 1];
        st = score_all_impl<float>(q, X[i], n, p->m, ldx, scores[i], what, p->slot_streams[j], who);
        if (st == GS_OK &&
            (e = hipMemcpyAsync(p->d_many_status + i, q->d_status, sizeof(int),
                                hipMemcpyDeviceToDevice, p->slot_streams[j])) != hipSuccess)
            st = hip_fail(e, "status copy");
    }
    // join, also after an error: the caller's stream waits for whatever was enqueued
    for (int j = 0; j < in_flight; ++j)
        if ((e = hipEventRecord(p->slot_join[j], p->slot_streams[j])) != hipSuccess ||
            (e = hipStreamWaitEvent(s, p->slot_join[j], 0)) != hipSuccess)
            return hip_fail(e, "stream join");
    p->many_count = st == GS_OK ? count : 0;
    return st;
}

int gs_many_status(gs_plan_t *p, int *status) {
    if (!p || !status) return fail(GS_EINVAL, "gs_many_status: NULL argument");
    if (p->many_count == 0)
        return fail(GS_EINVAL, "gs_many_status: no completed gs_score_all_many call on this plan");
    hipError_t e;
    for (hipEvent_t j : p->slot_join)
        if ((e = hipEventSynchronize(j)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    std::vector<int> flags(size_t(p->many_count));
    if ((e = hipMemcpy(flags.data(), p->d_many_status, flags.size() * sizeof(int),
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "status copy");
    int first = GS_OK;
    for (size_t i = 0; i < flags.size(); ++i) {
        const int f = flags[i];
        status[i] = (f & GS_FLAG_NOTFINITE) ? GS_ENOTFINITE
                    : (f & GS_FLAG_RANK)    ? GS_ERANK
                    : (f & GS_FLAG_RANGE)   ? GS_ERANGE
                                            : GS_OK;
        if (status[i] != GS_OK && first == GS_OK) {
            first = status[i];
            set_error("gs_many_status: dataset " + std::to_string(i) + " has status " +
                      std::to_string(first));
        }
    }
    return first;
}

int gs_qr_r0(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx, double *R0,
             void *stream) {
    int st = check_common(p, X, n, m, ldx, R0, "gs_qr_r0");
    if (st != GS_OK) return st;
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    p->front_x = nullptr;  // R0 is formed again, the anchors are not
    hipError_t e = launch_front_reset(p->d_status, p->d_stats, 1, s);
    if (e != hipSuccess) return hip_fail(e, "status reset launch");
    if ((e = launch_qr_r0(X, n, m, ldx, p->d_r0, R0, p->d_qr_a, p->d_qr_b, p->d_status, p->d_stats,
                          s)) != hipSuccess)
        return hip_fail(e, "R0 QR launch");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return GS_OK;
}

int gs_score_all(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx, float *scores,
                 int what, void *stream) {
    return score_all_impl<float>(p, X, n, m, ldx, scores, what, stream, "gs_score_all");
}

int gs_count_writes(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx,
                    uint32_t *counts, void *stream) {
    int st = check_common(p, X, n, m, ldx, counts, "gs_count_writes");
    if (st != GS_OK) return st;
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((st = front_half<float>(p, X, n, m, ldx, s, nullptr)) != GS_OK) return st;
    hipError_t e = launch_walk_count(p, static_cast<const float *>(p->d_anchor),
                                     static_cast<const float *>(p->d_tail), counts, n, s);
    if (e != hipSuccess) return hip_fail(e, "walk launch");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->last_stream = s;
    return GS_OK;
}

int gs_score_reduce(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx,
                    const gs_reduce_t *out, void *stream) {
    if (!out) return fail(GS_EINVAL, "gs_score_reduce: out is NULL");
    int st = check_common(p, X, n, m, ldx, out->best_score, "gs_score_reduce");
    if (st != GS_OK) return st;
    if (!out->best_parents || !out->logsumexp)
        return fail(GS_EINVAL, "gs_score_reduce: NULL output array");
    if (out->top_k < 0 || out->top_k > GS_REDUCE_MAX_TOPK)
        return fail(GS_EINVAL, "gs_score_reduce: top_k must be in 0..8");
    if (out->top_k > 0 && (!out->top_score || !out->top_parents))
        return fail(GS_EINVAL, "gs_score_reduce: top_k > 0 needs top_score and top_parents");
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    if (!p->red.pmin) {
        const size_t cnt = size_t(p->m) * size_t(p->nseg);
        hipError_t e;
        if ((e = hipMalloc(&p->red.pmin, cnt * 4)) != hipSuccess ||
            (e = hipMalloc(&p->red.pmask, cnt * 4)) != hipSuccess ||
            (e = hipMalloc(&p->red.psum, cnt * 4)) != hipSuccess ||
            (e = hipMalloc(&p->red.ptopv, cnt * GS_REDUCE_TOPK * 4)) != hipSuccess ||
            (e = hipMalloc(&p->red.ptopm, cnt * GS_REDUCE_TOPK * 4)) != hipSuccess ||
            (e = hipMalloc(&p->red.stage, size_t(p->m) * GS_REDUCE_SPLIT * sizeof(ReduceStage))) !=
                hipSuccess) {
            (void)hipFree(p->red.pmin);
            (void)hipFree(p->red.pmask);
            (void)hipFree(p->red.psum);
            (void)hipFree(p->red.ptopv);
            (void)hipFree(p->red.ptopm);
            p->red = ReducePartials{};
            return fail(GS_ENOMEM, std::string("reduction workspace: ") + hipGetErrorString(e));
        }
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t *ev = new_event_set(p);
    if ((st = front_half<float>(p, X, n, m, ldx, s, ev)) != GS_OK) return st;
    const bool top = out->top_k > 0;
    hipError_t e = launch_walk_reduce(p, static_cast<const float *>(p->d_anchor),
                                      static_cast<const float *>(p->d_tail), p->red, top, n, s);
    if (e != hipSuccess) return hip_fail(e, "reduce walk launch");
    if ((e = launch_reduce_children(p, p->red, top, out->best_score, out->best_parents,
                                    out->logsumexp, out->top_score, out->top_parents, out->top_k,
                                    s)) != hipSuccess)
        return hip_fail(e, "child merge launch");
    if (ev && (e = hipEventRecord(ev[3], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->last_stream = s;
    return GS_OK;
}

int gs_score_beta(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx, double *beta,
                  void *stream) {
    int st = check_common(p, X, n, m, ldx, beta, "gs_score_beta");
    if (st != GS_OK) return st;
    if (m > GS_BETA_MAX_M) return fail(GS_EINVAL, "gs_score_beta: m must be at most 22");
    if ((st = ensure_workspace(p, n)) != GS_OK) return st;
    const int k = m < 10 ? m : 10;
    hipError_t e;
    if (!p->d_ups || p->beta_k != k) {
        std::vector<int> seq;
        upsilon0(k, seq);
        std::vector<int8_t> s8(seq.begin(), seq.end());
        (void)hipFree(p->d_ups);
        p->d_ups = nullptr;
        if ((e = hipMalloc(&p->d_ups, std::max<size_t>(s8.size(), 1))) != hipSuccess)
            return fail(GS_ENOMEM, std::string("coefficient walk program: ") + hipGetErrorString(e));
        if (!s8.empty() &&
            (e = hipMemcpy(p->d_ups, s8.data(), s8.size(), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "coefficient walk program upload");
        p->beta_k = k;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    p->front_x = nullptr;  // R0 is formed again, the anchors are not
    if ((e = launch_front_reset(p->d_status, p->d_stats, 1, s)) != hipSuccess)
        return hip_fail(e, "status reset launch");
    if ((e = launch_qr_r0(X, n, m, ldx, p->d_r0, nullptr, p->d_qr_a, p->d_qr_b, p->d_status,
                          p->d_stats, s)) != hipSuccess)
        return hip_fail(e, "R0 QR launch");
    const int64_t nups = (int64_t(1) << k) - k - 1;
    if ((e = launch_beta_walk(p->d_r0, p->d_stats, m, k, p->d_ups, nups, beta, s)) != hipSuccess)
        return hip_fail(e, "coefficient walk launch");
    if ((e = hipEventRecord(p->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->last_stream = s;
    return GS_OK;
}

int gs_score_all_f64(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx, double *scores,
                     int what, void *stream) {
    return score_all_impl<double>(p, X, n, m, ldx, scores, what, stream, "gs_score_all_f64");
}

int gs_plan_workspace_bytes(const gs_plan_t *p, int64_t n, int backward, int64_t *bytes) {
    if (!p || !bytes) return fail(GS_EINVAL, "gs_plan_workspace_bytes: NULL argument");
    if (n <= p->m) return fail(GS_EINVAL, "gs_plan_workspace_bytes: need n > m");
    *bytes = workspace_bytes(p, n, backward != 0);
    return GS_OK;
}

int gs_sync_status(gs_plan_t *p) {
    if (!p) return fail(GS_EINVAL, "gs_sync_status: plan is NULL");
    if (p->device < 0) return GS_OK;
    hipError_t e = hipEventSynchronize(p->done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    int flags = 0;
    if ((e = hipMemcpy(&flags, p->d_status, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "status copy");
    if (flags & GS_FLAG_NOTFINITE) return fail(GS_ENOTFINITE, "X holds NaN or Inf");
    if (flags & GS_FLAG_RANK)
        return fail(GS_ERANK, "X is (numerically) rank deficient: a column lies within an angle "
                              "of n*eps of the span of the others");
    if (flags & GS_FLAG_RANGE)
        return fail(GS_ERANGE, "an RSS value lies outside the normal range of the output type");
    return GS_OK;
}

int gs_column_vif(gs_plan_t *p, double *vif) {
    if (!p || !vif) return fail(GS_EINVAL, "gs_column_vif: NULL argument");
    if (p->device < 0) return fail(GS_EINVAL, "gs_column_vif: the plan has not been used yet");
    hipError_t e = hipEventSynchronize(p->done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    const char *src = reinterpret_cast<const char *>(p->d_stats) + offsetof(ColStats, vif);
    if ((e = hipMemcpy(vif, src, sizeof(double) * size_t(p->m),
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "statistics copy");
    return GS_OK;
}

int gs_set_timing(gs_plan_t *p, int enable) {
    if (!p) return fail(GS_EINVAL, "gs_set_timing: plan is NULL");
    for (auto &ev : p->events) {
        (void)hipEventSynchronize(ev[3]);
        for (auto e : ev) (void)hipEventDestroy(e);
    }
    p->events.clear();
    p->timing = enable != 0;
    return GS_OK;
}

int gs_get_timing(gs_plan_t *p, double *ms, int64_t *count) {
    if (!p || !ms || !count) return fail(GS_EINVAL, "gs_get_timing: NULL argument");
    double acc[4] = {0, 0, 0, 0};
    int64_t cnt = 0;
    for (auto &ev : p->events) {
        hipError_t e = hipEventSynchronize(ev[3]);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        float t01 = 0, t12 = 0, t23 = 0, t03 = 0;
        if ((e = hipEventElapsedTime(&t01, ev[0], ev[1])) != hipSuccess ||
            (e = hipEventElapsedTime(&t12, ev[1], ev[2])) != hipSuccess ||
            (e = hipEventElapsedTime(&t23, ev[2], ev[3])) != hipSuccess ||
            (e = hipEventElapsedTime(&t03, ev[0], ev[3])) != hipSuccess)
            return hip_fail(e, "hipEventElapsedTime");
        acc[0] += t01;
        acc[1] += t12;
        acc[2] += t23;
        acc[3] += t03;
        ++cnt;
    }
    for (int i = 0; i < 4; ++i) ms[i] = cnt ? acc[i] / double(cnt) : 0.0;
    *count = cnt;
    return GS_OK;
}

}  // extern "C"
