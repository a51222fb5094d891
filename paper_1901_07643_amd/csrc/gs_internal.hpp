// Internal declarations of libgivscore: the plan object and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/givscore.h"
#include "walk_program.hpp"

// Device status word bits (OR-ed by kernels).
#define GS_FLAG_NOTFINITE 1
#define GS_FLAG_RANK 2

struct gs_plan_s {
    int m = 0, k = 0, ks = 0, q = 0;
    int64_t nseg = 0, nsub = 0;
    std::vector<uint32_t> prog;  // 2 words per sub-walk (layout in walk_program.hpp)

    // device workspace, allocated on first use on `device`
    int device = -1;
    uint32_t *d_prog = nullptr;
    double *d_r0 = nullptr;      // m x m
    double *d_qr_a = nullptr;    // TSQR ping-pong buffers
    double *d_qr_b = nullptr;
    int64_t qr_cap = 0;          // elements per TSQR buffer
    double *d_anchor = nullptr;  // nseg x k x 32
    double *d_tail = nullptr;    // nseg x 32
    int *d_status = nullptr;
    hipStream_t last_stream = nullptr;
    hipEvent_t done = nullptr;

    bool timing = false;
    std::vector<std::array<hipEvent_t, 4>> events;
};

namespace gs {

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Host planner (plan.cpp)
int build_program(gs_plan_s *p);

// Kernel launchers (return hipError_t of the launch)
// TSQR of X (n x m, row stride ldx) into R0 (m x m, upper, non-negative diagonal).
hipError_t launch_qr_r0(const double *X, int64_t n, int m, int64_t ldx, double *R0, double *bufA,
                        double *bufB, int *status, hipStream_t s);
int64_t qr_workspace_elems(int64_t n, int m);

// Segment anchors: FP64 R blocks of every segment from R0.
hipError_t launch_anchors(const double *R0, int m, int k, int ks, int64_t nseg, double *anchor,
                          double *tail, hipStream_t s);

// The walk.  T = float or double; writes the full table.
hipError_t launch_walk_f32(const gs_plan_s *p, const double *anchor, const double *tail, float *out,
                           int64_t n, bool bic, hipStream_t s);
hipError_t launch_walk_f64(const gs_plan_s *p, const double *anchor, const double *tail,
                           double *out, int64_t n, bool bic, hipStream_t s);

}  // namespace gs
