// rt_internal.h -- layouts shared by the kernels and the host code of the
// library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rtsort.h"

namespace rt {

constexpr int kMaxPasses = RT_MAX_PASSES;
constexpr int kMaxBits = RT_MAX_DIGIT_BITS;
constexpr int kMaxRadix = 1 << kMaxBits;

// Source/destination of one executed counting-sort pass.  Written on the
// device by the planning kernel once the histograms are known, so that pass
// skipping and the choice of ping-pong buffers need no host round trip.
struct PassPlan {
    const uint32_t *src_k;
    const uint32_t *src_v;
    uint32_t *dst_k;
    uint32_t *dst_v;
    uint32_t active;  // 0: pass skipped (its digit is constant)
    uint32_t shift;
    uint32_t width;
    uint32_t pad;
};

struct SortPlan {
    PassPlan pass[kMaxPasses];
    uint32_t executed;   // number of active passes
    uint32_t copy_back;  // 1: one pass ran, result sits in temp 1
    uint32_t pad[2];
};

// Host description of a sort handed to the planning kernel.
struct PlanArgs {
    uint32_t num_passes;
    uint32_t shift[kMaxPasses];
    uint32_t width[kMaxPasses];
    uint32_t no_skip;
    uint32_t n;
    uint32_t *user_k;
    uint32_t *user_v;
    uint32_t *t1_k;
    uint32_t *t1_v;
    uint32_t *t2_k;
    uint32_t *t2_v;
};

}  // namespace rt
