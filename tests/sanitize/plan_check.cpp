// Host planner under AddressSanitizer and UndefinedBehaviorSanitizer (test
// infrastructure, built with g++ by tests/test_sanitizers.py; no GPU involved).
// Builds plans over the whole range of sizes, checks the exactly-once coverage of the
// walk simulation, the swap sequence lengths and the argument checks.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../include/givscore.h"
#include "../../paper_1901_07643_amd/csrc/gs_internal.hpp"

// gs_plan_destroy lives with the device code; a plan that never ran on a device owns
// host memory only, which is all that is freed here.
extern "C" void gs_plan_destroy(gs_plan_t *p) { delete p; }

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

int main() {
    for (int m = 1; m <= 12; ++m) {
        const int64_t N = gs_num_families(m);
        CHECK(N == (int64_t(m) << (m - 1)));
        for (int ks = 1; ks <= 6 && ks <= m; ++ks)
            for (int k = ks; k <= m && k - ks <= 16; ++k) {
                gs_plan_t *p = nullptr;
                CHECK(gs_plan_tuned(m, k, ks, &p) == GS_OK);
                if (!p) continue;
                std::vector<int32_t> counts(size_t(N), 0);
                CHECK(gs_plan_count_emissions(p, counts.data(), N) == GS_OK);
                for (int64_t i = 0; i < N; ++i) CHECK(counts[size_t(i)] == 1);
                gs_plan_info_t info;
                CHECK(gs_plan_get_info(p, &info) == GS_OK);
                CHECK(info.swaps_per_segment == (int64_t(1) << k) - k - 1);
                gs_plan_destroy(p);
            }
    }
    // default plans up to the largest size (host work only)
    for (int m = 13; m <= GS_MAX_M; ++m) {
        gs_plan_t *p = nullptr;
        CHECK(gs_plan(m, &p) == GS_OK);
        gs_plan_destroy(p);
    }
    for (int m = 1; m <= 20; ++m) {
        const int64_t len = gs_upsilon(m, nullptr, 0);
        CHECK(len == (int64_t(1) << m) - m - 1);
        std::vector<int32_t> seq(size_t(len > 0 ? len : 1));
        CHECK(gs_upsilon(m, seq.data(), len) == len);
        for (int64_t i = 0; i < len; ++i) CHECK(seq[size_t(i)] >= 1 && seq[size_t(i)] < m);
    }
    // argument errors
    gs_plan_t *p = nullptr;
    CHECK(gs_plan(0, &p) != GS_OK);
    CHECK(gs_plan(GS_MAX_M + 1, &p) != GS_OK);
    CHECK(gs_plan_tuned(10, 3, 5, &p) != GS_OK);
    CHECK(gs_plan_tuned(10, 10, 7, &p) != GS_OK);
    CHECK(gs_family_index(5, 2, 0x4) == -1);
    CHECK(gs_family_index(5, 5, 0) == -1);
    CHECK(gs_upsilon(25, nullptr, 0) < 0);
    std::printf("planner checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
