// Launch interfaces of the element-wise and tensor-scalar kernels
// (elementwise.hip). Every pointer is device memory.
#pragma once

#include "common.h"

namespace pasta {

constexpr int kEwAdd = 0, kEwSub = 1, kEwMul = 2, kEwDiv = 3;  // pasta_ewop values

// z[i] = x[i] op y[i] for i < n, or z[i] = x[i] op s when y is null.
hipError_t launch_ew(int op, const float *x, const float *y, float s, float *z, uint64_t n, hipStream_t st);

struct TewInds {
    const uint32_t *p[kMaxOrder];
};
struct TewOut {
    uint32_t *p[kMaxOrder];
};

// The sorted concatenation of X then Y (perm[p] < nx: from X) has run heads
// head[p] and their exclusive scan run_of[p]. For each run r: run_val[r] =
// the combined value, run_pos[r] = its first position, run_keep[r] = 1 if the
// run is part of the result.
hipError_t launch_tew_runs(const uint32_t *head, const uint32_t *run_of, const uint32_t *perm, const float *vals,
                           uint64_t n, uint64_t nx, int op, float *run_val, uint32_t *run_pos, uint32_t *run_keep,
                           hipStream_t st);
// Kept runs to out / vals_out at out_of[r] (exclusive scan of run_keep);
// *count = number of kept runs.
hipError_t launch_tew_emit(const TewInds &sorted, uint32_t order, const uint32_t *run_pos, const float *run_val,
                           const uint32_t *run_keep, const uint32_t *out_of, uint64_t nruns, const TewOut &out,
                           float *vals_out, uint32_t *count, hipStream_t st);

}  // namespace pasta
