// Host planner of libgivscore: integer work only, done once per plan.
//
// Segments (Sec. 6): the m - k highest labels are each fixed either in front of
// the walked block (they are always parents) or behind it (never parents); each
// of the 2^(m-k) choices is an independent segment that starts from its own R
// and walks k variables.  Alg. 2 builds the same split from a processor's binary
// code; here the code bit is 1 for "front".
//
// Inside a segment the k walked variables are split into an inner block (the
// lowest ks labels) and q = k - ks middle variables.  The middle variables are
// walked by the paper's sequence Upsilon(q); the inner block Z sits between the
// middle variables that are currently in the prefix (front) and the others.
// A middle swap at p is followed by one crossing of Z by one middle variable, so
// that Z always follows exactly the new prefix set: consecutive entries of
// Upsilon differ by one, which keeps Z away from the pair being swapped.  At every
// resting point the inner block is walked by Upsilon(ks).  The number of Givens
// steps is (2^q - 1) ks + (2^q - q - 1) + 2^q (2^ks - ks - 1) = 2^k - k - 1, the
// optimum of Sec. 4, and every table line of 2^ks consecutive entries is produced
// by one inner walk.
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gs_internal.hpp"

namespace gs {

constexpr int kDefaultMaxK = 13;

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return GS_EHIP;
}

void upsilon0(int q, std::vector<int> &seq) {
    seq.clear();
    if (q >= 2) seq.push_back(0);
    for (int kk = 3; kk <= q; ++kk) {
        const size_t old = seq.size();
        for (int t = kk - 2; t >= 0; --t) seq.push_back(t);
        for (size_t t = 0; t < old; ++t) seq.push_back(seq[t] + 1);
    }
}

int build_program(gs_plan_s *p) {
    const int q = p->q, ks = p->ks;
    p->nsub = int64_t(1) << q;
    p->prog.assign(size_t(2 * p->nsub), 0u);
    std::vector<int> mu(q);
    for (int i = 0; i < q; ++i) mu[i] = ks + i;
    int z = q;
    uint32_t omask = (q == 0) ? 0u : ((1u << q) - 1u);
    auto put = [&](int64_t t, uint32_t w1, uint32_t moved = 0) {
        p->prog[2 * t] = omask | (uint32_t(z) << 16) | (moved << 21);
        p->prog[2 * t + 1] = w1;
    };
    put(0, 0u);
    int64_t t = 1;
    // Z starts behind every middle variable; move it to the front one variable at
    // a time: these are the prefixes of the initial middle ordering.
    for (int step = 0; step < q; ++step) {
        const int v = mu[z - 1];
        uint32_t w1 = SubWord::kHasTransition | (uint32_t(v) << 16) | (uint32_t(z) << 24);
        omask &= ~(1u << (v - ks));
        --z;
        put(t++, w1);
    }
    std::vector<int> seq;
    upsilon0(q, seq);
    for (int j : seq) {
        if (z == j + 1) return fail(GS_EINVAL, "planner: inner block between swapped pair");
        uint32_t w1 = SubWord::kHasTransition | SubWord::kHasMid | (uint32_t(j) << 2) |
                      (uint32_t(mu[j + 1]) << 8) | (uint32_t(z) << 24);
        const uint32_t moved = uint32_t(mu[j]);
        std::swap(mu[j], mu[j + 1]);
        if (z == j) {
            const int v = mu[z];
            w1 |= SubWord::kCrossLeft | (uint32_t(v) << 16);
            omask |= 1u << (v - ks);
            ++z;
        } else if (z == j + 2) {
            const int v = mu[z - 1];
            w1 |= uint32_t(v) << 16;
            omask &= ~(1u << (v - ks));
            --z;
        } else {
            return fail(GS_EINVAL, "planner: swap not adjacent to the inner block");
        }
        put(t++, w1, moved);
    }
    if (t != p->nsub) return fail(GS_EINVAL, "planner: wrong number of sub-walks");
    return GS_OK;
}

// Pack the segments into 64-lane waves.  Segment s walks k + b(s) columns (b(s)
// back variables); every segment runs the same program, so a wave costs the same
// whatever it holds and the aim is few waves.  Best-fit decreasing by width.
int pack_waves(gs_plan_s *p) {
    const int k = p->k, nout = p->m - p->k;
    std::vector<std::vector<int64_t>> by_width(nout + 1);
    for (int64_t s = 0; s < p->nseg; ++s) {
        const int b = nout - __builtin_popcountll((unsigned long long)s);
        by_width[b].push_back(s);
    }
    struct Bin {
        int used = 0;
        std::vector<int64_t> segs;
    };
    std::vector<Bin> bins;
    std::vector<std::vector<int>> by_free(65);  // bins indexed by free lanes
    for (int b = nout; b >= 0; --b) {
        const int w = k + b;
        if (w > 64) return fail(GS_EINVAL, "planner: segment wider than a wave");
        for (int64_t s : by_width[b]) {
            int pick = -1;
            for (int f = w; f <= 64 && pick < 0; ++f)
                if (!by_free[f].empty()) {
                    pick = by_free[f].back();
                    by_free[f].pop_back();
                }
            if (pick < 0) {
                pick = int(bins.size());
                bins.emplace_back();
            }
            Bin &bn = bins[pick];
            bn.segs.push_back(s);
            bn.used += w;
            by_free[64 - bn.used].push_back(pick);
        }
    }
    p->nwaves = int64_t(bins.size());
    p->lane_seg.assign(size_t(p->nwaves) * 64, -1);
    p->lane_loc.assign(size_t(p->nwaves) * 64, 0);
    for (size_t wv = 0; wv < bins.size(); ++wv) {
        int off = 0;
        for (int64_t s : bins[wv].segs) {
            const int w = k + nout - __builtin_popcountll((unsigned long long)s);
            for (int l = 0; l < w; ++l) {
                p->lane_seg[wv * 64 + off + l] = int32_t(s);
                p->lane_loc[wv * 64 + off + l] = int8_t(l);
            }
            off += w;
        }
    }
    return GS_OK;
}

// The walked block's ordering and the inner block's position after the last sub-walk:
// the state a replay of the whole walk ends in (the reverse walk of the adjoint starts
// there).  The same for every segment.
template <int KS>
static void walk_end_state(gs_plan_s *p) {
    constexpr auto &P = kInner<KS>;
    constexpr int N = InnerProgram<KS>::N;
    const int k = p->k, q = p->q;
    std::vector<int> order(static_cast<size_t>(k));
    for (int i = 0; i < q; ++i) order[size_t(i)] = KS + i;
    for (int i = 0; i < KS; ++i) order[size_t(q + i)] = i;
    int z = q;
    for (int64_t t = 0; t < p->nsub; ++t) {
        const uint32_t w1 = p->prog[size_t(2 * t + 1)];
        const bool fwd = (t & 1) == 0;
        if (w1 & SubWord::kHasTransition) {
            if (w1 & SubWord::kHasMid) {
                const int j = int((w1 >> 2) & 31);
                const int pos = j < z ? j : j + KS;
                std::swap(order[size_t(pos)], order[size_t(pos + 1)]);
            }
            if (w1 & SubWord::kCrossLeft) {  // the first middle variable behind moves in front
                const int v = order[size_t(z + KS)];
                for (int i = z + KS; i > z; --i) order[size_t(i)] = order[size_t(i - 1)];
                order[size_t(z)] = v;
                ++z;
            } else {  // the last middle variable in front moves behind
                const int v = order[size_t(z - 1)];
                for (int i = z - 1; i < z - 1 + KS; ++i) order[size_t(i)] = order[size_t(i + 1)];
                order[size_t(z - 1 + KS)] = v;
                --z;
            }
        }
        for (int st = 0; st < N; ++st) {
            const int j = fwd ? P.j_f[st] : P.j_r[st];
            std::swap(order[size_t(z + j)], order[size_t(z + j + 1)]);
        }
    }
    for (int i = 0; i < 32; ++i) p->end.order[i] = int8_t(i < k ? order[size_t(i)] : -1);
    p->end.z = z;
}

static void walk_end_state_ks(gs_plan_s *p) {
    switch (p->ks) {
        case 1: walk_end_state<1>(p); break;
        case 2: walk_end_state<2>(p); break;
        case 3: walk_end_state<3>(p); break;
        case 4: walk_end_state<4>(p); break;
        case 5: walk_end_state<5>(p); break;
        case 6: walk_end_state<6>(p); break;
        default: break;
    }
}

// ---- host simulation of a plan (for gs_plan_count_emissions) -------------------

template <int KS>
static int simulate(const gs_plan_s *p, int32_t *counts, int64_t len) {
    constexpr auto &P = kInner<KS>;
    constexpr int N = InnerProgram<KS>::N;
    const int m = p->m, k = p->k, q = p->q, ks = KS;
    const int nout = m - k;
    auto index_of = [&](int c, uint64_t S) -> int64_t {
        const uint64_t low = S & ((uint64_t(1) << c) - 1);
        const uint64_t high = (S >> (c + 1)) << c;
        return (int64_t(c) << (m - 1)) + int64_t(low | high);
    };
    // segments in the order the packed waves hold them; each must occupy consecutive
    // lanes with slots 0..width-1 and appear in exactly one wave
    std::vector<int64_t> seg_list;
    std::vector<char> seen(size_t(p->nseg), 0);
    for (int64_t wv = 0; wv < p->nwaves; ++wv) {
        int x = 0;
        while (x < 64) {
            const int32_t sg = p->lane_seg[size_t(wv * 64 + x)];
            if (sg < 0) {
                ++x;
                continue;
            }
            if (sg >= p->nseg || seen[size_t(sg)]) return fail(GS_EINVAL, "simulate: packing");
            seen[size_t(sg)] = 1;
            const int w = k + nout - __builtin_popcountll((unsigned long long)sg);
            if (x + w > 64) return fail(GS_EINVAL, "simulate: segment crosses a wave");
            for (int l = 0; l < w; ++l)
                if (p->lane_seg[size_t(wv * 64 + x + l)] != sg ||
                    p->lane_loc[size_t(wv * 64 + x + l)] != l)
                    return fail(GS_EINVAL, "simulate: segment lanes");
            seg_list.push_back(sg);
            x += w;
        }
    }
    if (int64_t(seg_list.size()) != p->nseg) return fail(GS_EINVAL, "simulate: missing segment");
    std::vector<int> order(k), backs;
    for (int64_t s : seg_list) {
        uint64_t F = 0;
        backs.clear();
        for (int b = 0; b < nout; ++b) {
            if ((s >> b) & 1) F |= uint64_t(1) << (k + b);
            else backs.push_back(k + b);
        }
        for (int i = 0; i < q; ++i) order[i] = ks + i;
        for (int i = 0; i < ks; ++i) order[q + i] = i;
        auto emit_prefix = [&](int plen) -> int {
            uint64_t S = F;
            for (int i = 0; i < plen; ++i) S |= uint64_t(1) << order[i];
            for (int i = plen; i < k; ++i) {
                const int64_t id = index_of(order[i], S);
                if (id < 0 || id >= len) return -1;
                counts[id] += 1;
            }
            for (int c : backs) {
                const int64_t id = index_of(c, S);
                if (id < 0 || id >= len) return -1;
                counts[id] += 1;
            }
            return 0;
        };
        int z = q;
        for (int64_t t = 0; t < p->nsub; ++t) {
            const uint32_t w0 = p->prog[2 * t], w1 = p->prog[2 * t + 1];
            const bool fwd = (t & 1) == 0;
            if (w1 & SubWord::kHasTransition) {
                const int zb = int((w1 >> 24) & 31);
                if (zb != z) return fail(GS_EINVAL, "simulate: z mismatch");
                if (w1 & SubWord::kHasMid) {
                    const int j = int((w1 >> 2) & 31), piv = int((w1 >> 8) & 31);
                    if (j < 0 || j + 1 >= q) return fail(GS_EINVAL, "simulate: middle swap range");
                    const int pos = j < z ? j : j + ks;
                    if ((j < z) != (j + 1 < z)) return fail(GS_EINVAL, "simulate: straddle");
                    if (order[pos + 1] != piv) return fail(GS_EINVAL, "simulate: mid pivot");
                    if (order[pos] != int((w0 >> 21) & 31)) return fail(GS_EINVAL, "simulate: mid moved");
                    std::swap(order[pos], order[pos + 1]);
                }
                const int v = int((w1 >> 16) & 31);
                if (w1 & SubWord::kCrossLeft) {
                    if (z + ks >= k) return fail(GS_EINVAL, "simulate: cross-left past the block");
                    if (order[z + ks] != v) return fail(GS_EINVAL, "simulate: cross-left var");
                    for (int i = z + ks; i > z; --i) order[i] = order[i - 1];
                    order[z] = v;
                    ++z;
                } else {
                    if (z < 1) return fail(GS_EINVAL, "simulate: cross-right with empty front");
                    if (order[z - 1] != v) return fail(GS_EINVAL, "simulate: cross-right var");
                    for (int i = z - 1; i < z - 1 + ks; ++i) order[i] = order[i + 1];
                    order[z - 1 + ks] = v;
                    --z;
                }
            }
            if (int((w0 >> 16) & 31) != z) return fail(GS_EINVAL, "simulate: z word");
            uint32_t om = 0;
            for (int i = 0; i < z; ++i) {
                if (order[i] < ks) return fail(GS_EINVAL, "simulate: inner var in front");
                om |= 1u << (order[i] - ks);
            }
            if (om != (w0 & 0xFFFFu)) return fail(GS_EINVAL, "simulate: front set");
            for (int i = 0; i < ks; ++i) {
                const int want = fwd ? P.order_f[i] : P.order_r[i];
                if (order[z + i] != want) return fail(GS_EINVAL, "simulate: inner order");
            }
            for (int pl = 0; pl <= ks; ++pl)
                if (emit_prefix(z + pl)) return fail(GS_EINVAL, "simulate: index range");
            for (int st = 0; st < N; ++st) {
                const int j = fwd ? P.j_f[st] : P.j_r[st];
                const int piv = fwd ? P.piv_f[st] : P.piv_r[st];
                if (order[z + j + 1] != piv) return fail(GS_EINVAL, "simulate: inner pivot");
                if (order[z + j] != (fwd ? P.mov_f[st] : P.mov_r[st]))
                    return fail(GS_EINVAL, "simulate: inner moved");
                std::swap(order[z + j], order[z + j + 1]);
                int mk = 0;
                for (int i = 0; i <= j; ++i) mk |= 1 << order[z + i];
                if (mk != (fwd ? P.mask_f[st] : P.mask_r[st]))
                    return fail(GS_EINVAL, "simulate: inner mask");
                if (emit_prefix(z + j + 1)) return fail(GS_EINVAL, "simulate: index range");
            }
        }
        // the state the adjoint's end-state anchors are formed in
        if (z != p->end.z) return fail(GS_EINVAL, "simulate: end position of the inner block");
        for (int i = 0; i < k; ++i)
            if (order[size_t(i)] != p->end.order[i]) return fail(GS_EINVAL, "simulate: end ordering");
    }
    return GS_OK;
}

}  // namespace gs

using namespace gs;

extern "C" {

int64_t gs_num_families(int m) {
    if (m < 1 || m > GS_MAX_M) return -1;
    return int64_t(m) << (m - 1);
}

int64_t gs_family_index(int m, int child, uint64_t parent_mask) {
    if (m < 1 || m > GS_MAX_M || child < 0 || child >= m) return -1;
    if ((parent_mask >> child) & 1u) return -1;
    if ((parent_mask >> m) != 0) return -1;
    const uint64_t low = parent_mask & ((uint64_t(1) << child) - 1);
    const uint64_t high = (parent_mask >> (child + 1)) << child;
    return (int64_t(child) << (m - 1)) + int64_t(low | high);
}

int64_t gs_upsilon(int m, int32_t *out, int64_t cap) {
    if (m < 1 || m > 24 || (cap > 0 && !out)) return fail(GS_EINVAL, "gs_upsilon: bad argument");
    std::vector<int> seq;
    upsilon0(m, seq);
    for (int64_t i = 0; i < cap && i < int64_t(seq.size()); ++i) out[i] = seq[i] + 1;
    return int64_t(seq.size());
}

int gs_plan_tuned(int m, int k, int ks, gs_plan_t **out) {
    if (!out) return fail(GS_EINVAL, "gs_plan: out is NULL");
    if (m < 1 || m > GS_MAX_M) return fail(GS_EINVAL, "gs_plan: m must be in 1..30");
    if (ks == 0) ks = m < 5 ? m : 5;
    if (k == 0) {
        // at least 2^13 segments when m allows (at m = 26, k = 13 leaves about 2.6
        // packed waves per SIMD; the walk is bound by its table writes, so fewer,
        // longer segments cost little there and halve the anchor work per step of
        // k), and at most 2^13 - 14 Givens steps per segment: the FP32 walk's
        // rounding error grows with the length of the walk from its FP64 start
        k = m - 13;
        if (k > kDefaultMaxK) k = kDefaultMaxK;
        if (k < ks) k = ks;
    }
    if (ks < 1 || ks > KS_MAX || ks > m) return fail(GS_EINVAL, "gs_plan: ks must be in 1..min(6,m)");
    if (k < ks || k > m || k - ks > Q_MAX)
        return fail(GS_EINVAL, "gs_plan: need ks <= k <= m and k - ks <= 16");
    gs_plan_s *p = new (std::nothrow) gs_plan_s();
    if (!p) return fail(GS_ENOMEM, "gs_plan: host allocation failed");
    static std::atomic<uint64_t> next_id{1};
    p->id = next_id.fetch_add(1);
    p->m = m;
    p->k = k;
    p->ks = ks;
    p->q = k - ks;
    p->nseg = int64_t(1) << (m - k);
    int st = build_program(p);
    if (st == GS_OK) walk_end_state_ks(p);
    if (st == GS_OK) st = pack_waves(p);
    if (st != GS_OK) {
        delete p;
        return st;
    }
    *out = p;
    return GS_OK;
}

int gs_plan(int m, gs_plan_t **out) { return gs_plan_tuned(m, 0, 0, out); }

int gs_plan_get_info(const gs_plan_t *p, gs_plan_info_t *info) {
    if (!p || !info) return fail(GS_EINVAL, "gs_plan_get_info: NULL argument");
    info->m = p->m;
    info->k = p->k;
    info->ks = p->ks;
    info->q = p->q;
    info->num_segments = p->nseg;
    info->sub_per_segment = p->nsub;
    info->swaps_per_segment = (int64_t(1) << p->k) - p->k - 1;
    info->num_families = int64_t(p->m) << (p->m - 1);
    info->num_waves = p->nwaves;
    return GS_OK;
}

int gs_plan_count_emissions(const gs_plan_t *p, int32_t *counts, int64_t len) {
    if (!p || !counts) return fail(GS_EINVAL, "gs_plan_count_emissions: NULL argument");
    if (p->m > 22) return fail(GS_EINVAL, "gs_plan_count_emissions: m > 22");
    if (len < (int64_t(p->m) << (p->m - 1))) return fail(GS_EINVAL, "gs_plan_count_emissions: len");
    switch (p->ks) {
        case 1: return simulate<1>(p, counts, len);
        case 2: return simulate<2>(p, counts, len);
        case 3: return simulate<3>(p, counts, len);
        case 4: return simulate<4>(p, counts, len);
        case 5: return simulate<5>(p, counts, len);
        case 6: return simulate<6>(p, counts, len);
        default: return fail(GS_EINVAL, "bad ks");
    }
}

const char *gs_last_error(void) { return g_err.c_str(); }

}  // extern "C"
