// gs_score_all_static: gs_score_all with its device workspace in a fixed, file-scope
// device array instead of memory allocated by the library, for callers that cannot
// allocate (code under graph capture, tight serving loops, harnesses that forbid it).
//
// The array `scratch` (GS_STATIC_SCRATCH_BYTES) exists once per device for the life
// of the process.  Its device address is looked up once per device with
// hipGetSymbolAddress (the array's name is only a host-side stand-in); every launch
// then gets pointers into it.  Layout of one call, each piece 256-byte aligned:
//   status word, column statistics, R0, walk program, packed lane tables, anchors and
//   tails (FP32), the two TSQR buffers.
// The walk program and lane tables are copied in from the plan (host memory) when the
// resident plan changes; every other piece is rewritten by each call.  All calls on
// one device share the array: calls that overlap on a device (different streams, no
// synchronisation) race and corrupt each other.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "gs_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[GS_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {};     // device address of `scratch` per device
uint64_t g_resident[kMaxDevices] = {};      // plan id whose tables the array holds

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

struct Layout {
    int64_t status, stats, r0, prog, lane_seg, lane_loc, anchor, tail, qr_a, qr_b, total;
};

Layout layout(const gs_plan_s *p, int64_t n) {
    Layout L;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t at = off;
        off += align256(bytes);
        return at;
    };
    L.status = take(16);
    L.stats = take(int64_t(sizeof(ColStats)));
    L.r0 = take(int64_t(p->m) * p->m * 8);
    L.prog = take(int64_t(p->prog.size()) * 4);
    L.lane_seg = take(int64_t(p->lane_seg.size()) * 4);
    L.lane_loc = take(int64_t(p->lane_loc.size()));
    L.anchor = take(p->nseg * p->k * 32 * 4);
    L.tail = take(p->nseg * 32 * 4);
    const int64_t qr = gs::qr_workspace_elems(n, p->m) * 8;
    L.qr_a = take(qr);
    L.qr_b = take(qr);
    L.total = off;
    return L;
}

// flags of the status word -> gs_status code, written to the caller's int
__global__ void status_code_kernel(const int *flags, int *code) {
    if (threadIdx.x != 0) return;
    const int f = flags[0];
    code[0] = (f & GS_FLAG_NOTFINITE) ? GS_ENOTFINITE
              : (f & GS_FLAG_RANK)    ? GS_ERANK
              : (f & GS_FLAG_RANGE)   ? GS_ERANGE
                                      : GS_OK;
}

}  // namespace

using namespace gs;

extern "C" int gs_score_all_static(gs_plan_t *p, const double *X, int64_t n, int m, int64_t ldx,
                                   float *scores, int what, int *status_code, void *stream) {
    if (!p) return fail(GS_EINVAL, "gs_score_all_static: plan is NULL");
    if (!X || !scores) return fail(GS_EINVAL, "gs_score_all_static: NULL data pointer");
    if (m != p->m) return fail(GS_EINVAL, "gs_score_all_static: m differs from the plan's m");
    if (n <= m) return fail(GS_EINVAL, "gs_score_all_static: need n > m samples");
    if (ldx < m) return fail(GS_EINVAL, "gs_score_all_static: ldx < m");
    if (reinterpret_cast<uintptr_t>(scores) % 16 != 0)
        return fail(GS_EINVAL, "gs_score_all_static: output must be 16-byte aligned");
    if (what != GS_OUT_BIC && what != GS_OUT_RSS)
        return fail(GS_EINVAL, "gs_score_all_static: what must be GS_OUT_BIC or GS_OUT_RSS");
    const Layout L = layout(p, n);
    if (L.total > int64_t(GS_STATIC_SCRATCH_BYTES))
        return fail(GS_ENOMEM, "gs_score_all_static: this plan and n need " +
                                   std::to_string(L.total) + " bytes of workspace; the static "
                                   "array holds " + std::to_string(int64_t(GS_STATIC_SCRATCH_BYTES)));
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GS_EINVAL, "gs_score_all_static: device index");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_ptr[dev]) {
            void *ptr = nullptr;
            if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
                return hip_fail(e, "hipGetSymbolAddress(scratch)");
            g_ptr[dev] = static_cast<unsigned char *>(ptr);
        }
        base = g_ptr[dev];
        if (g_resident[dev] != p->id) {
            if ((e = hipMemcpyAsync(base + L.prog, p->prog.data(), p->prog.size() * 4,
                                    hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(base + L.lane_seg, p->lane_seg.data(), p->lane_seg.size() * 4,
                                    hipMemcpyHostToDevice, s)) != hipSuccess ||
                (e = hipMemcpyAsync(base + L.lane_loc, p->lane_loc.data(), p->lane_loc.size(),
                                    hipMemcpyHostToDevice, s)) != hipSuccess) {
                g_resident[dev] = 0;
                return hip_fail(e, "plan table upload");
            }
            g_resident[dev] = p->id;
        }
    }
    int *status = reinterpret_cast<int *>(base + L.status);
    ColStats *stats = reinterpret_cast<ColStats *>(base + L.stats);
    double *r0 = reinterpret_cast<double *>(base + L.r0);
    float *anchor = reinterpret_cast<float *>(base + L.anchor);
    float *tail = reinterpret_cast<float *>(base + L.tail);
    if ((e = launch_front_reset(status, stats, 1, s)) != hipSuccess)
        return hip_fail(e, "status reset launch");
    if ((e = launch_qr_r0(X, n, m, ldx, r0, nullptr, reinterpret_cast<double *>(base + L.qr_a),
                          reinterpret_cast<double *>(base + L.qr_b), status, stats, s)) !=
        hipSuccess)
        return hip_fail(e, "R0 QR launch");
    if ((e = launch_anchors<float>(r0, stats, p->m, p->k, p->ks, p->nseg, anchor, tail, s)) !=
        hipSuccess)
        return hip_fail(e, "anchor launch");
    const WalkTables t{reinterpret_cast<const uint32_t *>(base + L.prog),
                       reinterpret_cast<const int32_t *>(base + L.lane_seg),
                       reinterpret_cast<const int8_t *>(base + L.lane_loc), status, stats};
    if ((e = launch_walk_f32_tables(p, t, anchor, tail, scores, n, what == GS_OUT_BIC, s)) !=
        hipSuccess)
        return hip_fail(e, "walk launch");
    if (status_code) {
        hipLaunchKernelGGL(status_code_kernel, dim3(1), dim3(64), 0, s, status, status_code);
        if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "status launch");
    }
    return GS_OK;
}
