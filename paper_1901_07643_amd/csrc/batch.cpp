// Batched scoring: many datasets of different sizes in one launch per stage.
//
// Every dataset gets its own plan (segments, walk program, packed waves).  The
// stages run once for the whole batch: the TSQR passes as one launch per pass over
// all (dataset, row block) jobs, the anchors as one launch over all segments, the
// walk as one launch over all waves, ordered longest walk first so that the short
// datasets fill in behind the long ones.  The sequence can be captured once into a
// hipGraph and replayed; the kernels read the datasets' pointers from a device
// table, so new data buffers only need a table update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "gs_internal.hpp"

using namespace gs;

struct gs_batch_s {
    int count = 0;
    std::vector<gs_plan_s *> plans;
    std::vector<int> m;
    std::vector<int64_t> n;
    int mmax = 0, qmax = 0;
    int64_t total_waves = 0, total_segs = 0, total_families = 0;

    // host tables
    std::vector<BatchItem> items;
    std::vector<int64_t> seg_prefix;
    std::vector<int32_t> wave_item, wave_local;
    std::vector<TsqrJob> jobs;  // all passes, concatenated
    std::vector<int> pass_off, pass_cnt;
    std::vector<int> pass0_job_item;  // for pass-0 jobs: dataset index (A = X of it)
    std::vector<size_t> prog_off, lane_off, r0_off, qr_off, qr_len, an_off, tl_off, eb_off;
    size_t prog_total = 0, lane_total = 0, r0_total = 0, qr_total = 0, an_total = 0, tl_total = 0,
           eb_total = 0;

    // device
    int device = -1;
    uint32_t *d_prog = nullptr;
    int32_t *d_lane_seg = nullptr;
    int8_t *d_lane_loc = nullptr;
    double *d_r0 = nullptr, *d_qr = nullptr;
    float *d_anchor = nullptr, *d_tail = nullptr;
    int *d_status = nullptr;
    int *d_eblk = nullptr;  // first-pass block exponents of every dataset
    ColStats *d_stats = nullptr;
    BatchItem *d_items = nullptr;
    int64_t *d_seg_prefix = nullptr;
    int32_t *d_wave_item = nullptr, *d_wave_local = nullptr;
    TsqrJob *d_jobs = nullptr;
    hipEvent_t done = nullptr;

    // data pointers the device tables hold
    std::vector<const double *> cur_x;
    std::vector<int64_t> cur_ldx;
    std::vector<float *> cur_out;
    bool tables_valid = false;

    // captured graphs, one per output kind
    hipStream_t cap = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
};

namespace {

void batch_free_device(gs_batch_s *b) {
    for (int w = 0; w < 2; ++w) {
        if (b->exec[w]) (void)hipGraphExecDestroy(b->exec[w]);
        if (b->graph[w]) (void)hipGraphDestroy(b->graph[w]);
        b->exec[w] = nullptr;
        b->graph[w] = nullptr;
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->done) (void)hipEventDestroy(b->done);
    b->cap = nullptr;
    b->done = nullptr;
    void *ptrs[] = {b->d_prog,   b->d_lane_seg, b->d_lane_loc,   b->d_r0,        b->d_qr,
                    b->d_anchor, b->d_tail,     b->d_status,     b->d_eblk,      b->d_stats,
                    b->d_items,  b->d_seg_prefix, b->d_wave_item, b->d_wave_local, b->d_jobs};
    for (void *p : ptrs) (void)hipFree(p);
    b->d_prog = nullptr;
    b->d_lane_seg = nullptr;
    b->d_lane_loc = nullptr;
    b->d_r0 = b->d_qr = nullptr;
    b->d_anchor = b->d_tail = nullptr;
    b->d_status = nullptr;
    b->d_eblk = nullptr;
    b->d_stats = nullptr;
    b->d_items = nullptr;
    b->d_seg_prefix = nullptr;
    b->d_wave_item = b->d_wave_local = nullptr;
    b->d_jobs = nullptr;
    b->device = -1;
    b->tables_valid = false;
}

template <typename P>
hipError_t alloc_copy(P **dst, const void *src, size_t bytes) {
    hipError_t e = hipMalloc(dst, bytes ? bytes : 16);
    if (e != hipSuccess) return e;
    if (bytes && src) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return e;
}

int batch_ensure_device(gs_batch_s *b) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (b->device >= 0) {
        if (b->device != dev) return fail(GS_EINVAL, "batch was first used on another device");
        return GS_OK;
    }
    b->device = dev;
    // concatenated programs and lane tables
    std::vector<uint32_t> prog(b->prog_total);
    std::vector<int32_t> lseg(b->lane_total * 64);
    std::vector<int8_t> lloc(b->lane_total * 64);
    for (int i = 0; i < b->count; ++i) {
        const gs_plan_s *p = b->plans[i];
        std::copy(p->prog.begin(), p->prog.end(), prog.begin() + b->prog_off[i]);
        std::copy(p->lane_seg.begin(), p->lane_seg.end(), lseg.begin() + b->lane_off[i] * 64);
        std::copy(p->lane_loc.begin(), p->lane_loc.end(), lloc.begin() + b->lane_off[i] * 64);
    }
    if ((e = alloc_copy(&b->d_prog, prog.data(), prog.size() * 4)) != hipSuccess ||
        (e = alloc_copy(&b->d_lane_seg, lseg.data(), lseg.size() * 4)) != hipSuccess ||
        (e = alloc_copy(&b->d_lane_loc, lloc.data(), lloc.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_r0, b->r0_total * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&b->d_qr, std::max<size_t>(b->qr_total, 1) * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&b->d_anchor, b->an_total * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&b->d_tail, b->tl_total * sizeof(float))) != hipSuccess ||
        (e = hipMalloc(&b->d_status, b->count * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&b->d_eblk, std::max<size_t>(b->eb_total, 1) * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&b->d_stats, b->count * sizeof(ColStats))) != hipSuccess ||
        (e = hipMalloc(&b->d_items, 2 * size_t(b->count) * sizeof(BatchItem))) != hipSuccess ||
        (e = alloc_copy(&b->d_seg_prefix, b->seg_prefix.data(), b->seg_prefix.size() * 8)) !=
            hipSuccess ||
        (e = alloc_copy(&b->d_wave_item, b->wave_item.data(), b->wave_item.size() * 4)) !=
            hipSuccess ||
        (e = alloc_copy(&b->d_wave_local, b->wave_local.data(), b->wave_local.size() * 4)) !=
            hipSuccess ||
        (e = hipMalloc(&b->d_jobs, std::max<size_t>(b->jobs.size(), 1) * sizeof(TsqrJob))) !=
            hipSuccess ||
        (e = hipMemset(b->d_status, 0, b->count * sizeof(int))) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess) {
        batch_free_device(b);
        return fail(GS_ENOMEM, std::string("batch workspace: ") + hipGetErrorString(e));
    }
    // device addresses of the per-dataset pieces
    for (int i = 0; i < b->count; ++i) {
        BatchItem &it = b->items[i];
        const gs_plan_s *p = b->plans[i];
        it.R0 = b->d_r0 + b->r0_off[i];
        it.anchor = b->d_anchor + b->an_off[i];
        it.tail = b->d_tail + b->tl_off[i];
        it.prog = b->d_prog + b->prog_off[i];
        it.lane_seg = b->d_lane_seg + b->lane_off[i] * 64;
        it.lane_loc = b->d_lane_loc + b->lane_off[i] * 64;
        it.status = b->d_status + i;
        it.stats = b->d_stats + i;
        (void)p;
    }
    // TSQR job pointers into the workspace (pass-0 inputs are filled with the data)
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        TsqrJob &jb = b->jobs[j];
        const int it = int(reinterpret_cast<intptr_t>(jb.status));  // dataset index, see create
        jb.status = b->d_status + it;
        jb.stats = b->d_stats + it;
        jb.eblk = b->d_eblk + b->eb_off[it];
        const intptr_t rtag = reinterpret_cast<intptr_t>(jb.Rout);
        const intptr_t atag = reinterpret_cast<intptr_t>(jb.A);
        // tags: Rout = -1 -> R0; otherwise offset+1 into d_qr; A = 0 -> X, else offset+1 into d_qr
        jb.Rout = rtag == -1 ? b->d_r0 + b->r0_off[it] : b->d_qr + (rtag - 1);
        jb.A = atag == 0 ? nullptr : b->d_qr + (atag - 1);
    }
    return GS_OK;
}

}  // namespace

extern "C" {

int gs_batch_create(int count, const int *m, const int64_t *n, const int *k, gs_batch_t **out) {
    if (!out || !m || !n || count < 1 || count > 4096)
        return fail(GS_EINVAL, "gs_batch_create: bad arguments");
    gs_batch_s *b = new (std::nothrow) gs_batch_s();
    if (!b) return fail(GS_ENOMEM, "gs_batch_create: host allocation");
    b->count = count;
    b->plans.assign(count, nullptr);
    b->m.assign(m, m + count);
    b->n.assign(n, n + count);
    for (int i = 0; i < count; ++i) {
        if (m[i] < BATCH_KS || m[i] > GS_MAX_M || n[i] <= m[i]) {
            gs_batch_destroy(b);
            return fail(GS_EINVAL, "gs_batch_create: dataset " + std::to_string(i) +
                                       " needs 5 <= m <= 30 and n > m");
        }
        int st = gs_plan_tuned(m[i], k ? k[i] : 0, BATCH_KS, &b->plans[i]);
        if (st != GS_OK) {
            gs_batch_destroy(b);
            return st;
        }
        b->mmax = std::max(b->mmax, m[i]);
    }
    // offsets
    b->items.resize(count);
    b->prog_off.resize(count);
    b->lane_off.resize(count);
    b->r0_off.resize(count);
    b->qr_off.resize(count);
    b->qr_len.resize(count);
    b->an_off.resize(count);
    b->tl_off.resize(count);
    b->eb_off.resize(count);
    b->seg_prefix.assign(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        const gs_plan_s *p = b->plans[i];
        b->prog_off[i] = b->prog_total;
        b->prog_total += p->prog.size();
        b->lane_off[i] = b->lane_total;
        b->lane_total += size_t(p->nwaves);
        b->r0_off[i] = b->r0_total;
        b->r0_total += size_t(p->m) * p->m;
        const int64_t nb0 = (n[i] + tsqr_rows_per_block() - 1) / tsqr_rows_per_block();
        b->qr_off[i] = b->qr_total;
        b->qr_len[i] = size_t(nb0) * p->m * p->m;
        b->qr_total += 2 * b->qr_len[i];
        b->eb_off[i] = b->eb_total;
        b->eb_total += size_t(nb0) * 32;
        b->an_off[i] = b->an_total;
        b->an_total += size_t(p->nseg) * p->k * 32;
        b->tl_off[i] = b->tl_total;
        b->tl_total += size_t(p->nseg) * 32;
        b->seg_prefix[i + 1] = b->seg_prefix[i] + p->nseg;
        b->total_families += int64_t(p->m) << (p->m - 1);
        BatchItem &it = b->items[i];
        std::memset(&it, 0, sizeof(it));
        it.m = p->m;
        it.k = p->k;
        it.ks = p->ks;
        it.q = p->q;
        it.nseg = p->nseg;
        it.nsub = p->nsub;
        it.nwaves = p->nwaves;
        b->qmax = std::max(b->qmax, p->q);
    }
    b->total_segs = b->seg_prefix[count];
    // waves, longest walk (most sub-walks) first
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        if (b->plans[a]->nsub != b->plans[c]->nsub) return b->plans[a]->nsub > b->plans[c]->nsub;
        return b->plans[a]->nwaves > b->plans[c]->nwaves;
    });
    for (int i : order)
        for (int64_t w = 0; w < b->plans[i]->nwaves; ++w) {
            b->wave_item.push_back(i);
            b->wave_local.push_back(int32_t(w));
        }
    b->total_waves = int64_t(b->wave_item.size());
    // TSQR passes (pointer fields hold tags until the device workspace exists)
    struct Cur {
        int64_t rows, lda;
        intptr_t src;  // 0 = X, else offset + 1 into the TSQR workspace
        int which;     // next destination buffer (0/1)
        bool done;
    };
    std::vector<Cur> cur(count);
    for (int i = 0; i < count; ++i) cur[i] = {n[i], -1, 0, 0, false};
    for (int pass = 0;; ++pass) {
        const int start = int(b->jobs.size());
        for (int i = 0; i < count; ++i) {
            if (cur[i].done) continue;
            const int mi = m[i];
            const int64_t nb = (cur[i].rows + tsqr_rows_per_block() - 1) / tsqr_rows_per_block();
            const bool final_pass = nb == 1;
            const intptr_t dst = final_pass ? -1
                                            : intptr_t(b->qr_off[i] + cur[i].which * b->qr_len[i]) + 1;
            for (int64_t blk = 0; blk < nb; ++blk) {
                TsqrJob jb;
                jb.A = reinterpret_cast<const double *>(cur[i].src);
                jb.nrows = cur[i].rows;
                jb.lda = cur[i].lda;
                jb.Rout = final_pass ? reinterpret_cast<double *>(intptr_t(-1))
                                     : reinterpret_cast<double *>(dst + blk * mi * mi);
                jb.status = reinterpret_cast<int *>(intptr_t(i));
                jb.stats = nullptr;
                jb.eblk = nullptr;
                jb.n_orig = n[i];
                jb.m = mi;
                jb.block = int(blk);
                jb.first = pass == 0;
                jb.rescale = pass == 1;
                jb.final_pass = final_pass;
                b->jobs.push_back(jb);
                b->pass0_job_item.push_back(pass == 0 ? i : -1);
            }
            if (final_pass) {
                cur[i].done = true;
            } else {
                cur[i].src = dst;
                cur[i].rows = nb * mi;
                cur[i].lda = mi;
                cur[i].which ^= 1;
            }
        }
        const int cnt = int(b->jobs.size()) - start;
        if (cnt == 0) break;
        b->pass_off.push_back(start);
        b->pass_cnt.push_back(cnt);
    }
    b->cur_x.assign(count, nullptr);
    b->cur_ldx.assign(count, 0);
    b->cur_out.assign(count, nullptr);
    *out = b;
    return GS_OK;
}

void gs_batch_destroy(gs_batch_t *b) {
    if (!b) return;
    if (b->device >= 0) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b->device);
        if (b->done) (void)hipEventSynchronize(b->done);
        batch_free_device(b);
        (void)hipSetDevice(cur);
    }
    for (gs_plan_s *p : b->plans) gs_plan_destroy(p);
    delete b;
}

int gs_batch_info(const gs_batch_t *b, int64_t *total_waves, int64_t *total_segments,
                  int64_t *total_families) {
    if (!b) return fail(GS_EINVAL, "gs_batch_info: NULL batch");
    if (total_waves) *total_waves = b->total_waves;
    if (total_segments) *total_segments = b->total_segs;
    if (total_families) *total_families = b->total_families;
    return GS_OK;
}

// One pass of the whole batch: status reset, TSQR passes, anchors, walk.  The item
// table for BIC comes first in d_items, the one for RSS second.
static hipError_t enqueue_batch(gs_batch_s *b, bool bic, hipStream_t s) {
    const BatchItem *items = b->d_items + (bic ? 0 : b->count);
    hipError_t e = launch_front_reset(b->d_status, b->d_stats, b->count, s);
    if (e != hipSuccess) return e;
    for (size_t p = 0; p < b->pass_off.size(); ++p)
        if ((e = launch_tsqr_batched(b->d_jobs + b->pass_off[p], b->pass_cnt[p], b->mmax, s)) != hipSuccess)
            return e;
    if ((e = launch_anchors_batched_f32(items, b->d_seg_prefix, b->count, b->total_segs,
                                        b->mmax, s)) != hipSuccess)
        return e;
    return launch_walk_batched_f32(items, b->d_wave_item, b->d_wave_local, b->total_waves, b->qmax,
                                   bic, s);
}

int gs_score_batched(gs_batch_t *b, const gs_batch_data_t *data, int what, int use_graph,
                     void *stream) {
    if (!b || !data) return fail(GS_EINVAL, "gs_score_batched: NULL argument");
    if (what != GS_OUT_BIC && what != GS_OUT_RSS)
        return fail(GS_EINVAL, "gs_score_batched: what must be GS_OUT_BIC or GS_OUT_RSS");
    for (int i = 0; i < b->count; ++i) {
        if (!data[i].X || !data[i].scores || data[i].ldx < b->m[i])
            return fail(GS_EINVAL, "gs_score_batched: bad data for dataset " + std::to_string(i));
        if (reinterpret_cast<uintptr_t>(data[i].scores) % 16 != 0)
            return fail(GS_EINVAL, "gs_score_batched: scores must be 16-byte aligned");
    }
    int st = batch_ensure_device(b);
    if (st != GS_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e;
    bool changed = !b->tables_valid;
    for (int i = 0; i < b->count && !changed; ++i)
        changed = data[i].X != b->cur_x[i] || data[i].ldx != b->cur_ldx[i] ||
                  data[i].scores != b->cur_out[i];
    if (changed) {
        // the previous call may still read the tables
        if ((e = hipEventSynchronize(b->done)) != hipSuccess) return hip_fail(e, "batch sync");
        std::vector<BatchItem> tab(2 * size_t(b->count));
        for (int i = 0; i < b->count; ++i) {
            b->cur_x[i] = data[i].X;
            b->cur_ldx[i] = data[i].ldx;
            b->cur_out[i] = data[i].scores;
            BatchItem it = b->items[i];
            it.out = data[i].scores;
            const double dn = double(b->n[i]);
            it.nlog = dn * 0.6931471805599453;  // the FP32 walk takes log2 in hardware
            it.lnn = std::log(dn);
            it.nln2 = dn * 0.6931471805599453;
            it.row_scale = 1.0 / std::sqrt(dn);  // BIC: the walk sees RSS / n
            tab[i] = it;
            it.row_scale = 1.0;  // RSS
            tab[b->count + i] = it;
        }
        for (size_t j = 0; j < b->jobs.size(); ++j)
            if (b->pass0_job_item[j] >= 0) {
                b->jobs[j].A = data[b->pass0_job_item[j]].X;
                b->jobs[j].lda = data[b->pass0_job_item[j]].ldx;
            }
        if ((e = hipMemcpy(b->d_jobs, b->jobs.data(), b->jobs.size() * sizeof(TsqrJob),
                           hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(b->d_items, tab.data(), tab.size() * sizeof(BatchItem),
                           hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "batch tables");
        b->tables_valid = true;
    }
    const bool bic = what == GS_OUT_BIC;
    if (use_graph) {
        const int w = bic ? 0 : 1;
        if (!b->exec[w]) {
            if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
                return hip_fail(e, "hipStreamBeginCapture");
            hipError_t le = enqueue_batch(b, bic, b->cap);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(b->cap, &g);
            if (le != hipSuccess) return hip_fail(le, "batch launch during capture");
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            b->graph[w] = g;
            if ((e = hipGraphInstantiate(&b->exec[w], g, nullptr, nullptr, 0)) != hipSuccess)
                return hip_fail(e, "hipGraphInstantiate");
        }
        if ((e = hipGraphLaunch(b->exec[w], s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        if ((e = enqueue_batch(b, bic, s)) != hipSuccess) return hip_fail(e, "batch launch");
    }
    if ((e = hipEventRecord(b->done, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    return GS_OK;
}

int gs_batch_status(gs_batch_t *b, int *status) {
    if (!b || !status) return fail(GS_EINVAL, "gs_batch_status: NULL argument");
    if (b->device < 0) {
        for (int i = 0; i < b->count; ++i) status[i] = GS_OK;
        return GS_OK;
    }
    hipError_t e = hipEventSynchronize(b->done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    std::vector<int> flags(b->count);
    if ((e = hipMemcpy(flags.data(), b->d_status, b->count * sizeof(int), hipMemcpyDeviceToHost)) !=
        hipSuccess)
        return hip_fail(e, "status copy");
    int worst = GS_OK;
    for (int i = 0; i < b->count; ++i) {
        status[i] = (flags[i] & GS_FLAG_NOTFINITE) ? GS_ENOTFINITE
                    : (flags[i] & GS_FLAG_RANK)    ? GS_ERANK
                    : (flags[i] & GS_FLAG_RANGE)   ? GS_ERANGE
                                                   : GS_OK;
        if (status[i] != GS_OK) worst = status[i];
    }
    return worst;
}

}  // extern "C"
