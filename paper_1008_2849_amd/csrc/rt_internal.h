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

// A pass splits its input into at most kChunks contiguous chunks, one per
// XCD of the MI355X, each with its own lookback chain and its own output
// start per digit.  The tiles of one chunk then run on one XCD, so the digit
// runs of neighbouring tiles, which share cache lines at their ends, are
// written through one L2 and leave it as whole lines.
constexpr int kChunks = 8;
constexpr int kChunkRadix = 256;  // row stride of the per-chunk tables (digits of at most 8 bits)
constexpr size_t kChunkMinItems = static_cast<size_t>(1) << 25;  // smaller sorts: one chain per pass

// Source/destination of one executed counting-sort pass.  Written on the
// device by the planning kernel once the histograms are known, so that pass
// skipping, the choice of ping-pong buffers and the chunks need no host
// round trip.
struct PassPlan {
    const uint32_t *src_k;
    const uint32_t *src_v;
    uint32_t *dst_k;
    uint32_t *dst_v;
    // cbase[x * kChunkRadix + d]: output slot of the first item of digit d
    // in chunk x (one row, of up to kMaxRadix digits, with one chunk)
    const uint32_t *cbase;
    uint32_t active;  // 0: pass skipped (its digit is constant)
    uint32_t shift;
    uint32_t width;
    uint32_t nchunks;              // 1 or kChunks
    uint32_t cstart[kChunks + 1];  // chunk x reads input items [cstart[x], cstart[x + 1])
    uint32_t ctile[kChunks + 1];   // lookback index of chunk x's first tile; ctile[nchunks] = all tiles
    uint32_t pad[2];
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
    uint32_t tile;                    // items per tile of the pass kernels
    uint32_t chunked;                 // histograms are per chunk (see k_histogram)
    uint32_t pos_bound[kChunks + 1];  // chunks of the first pass: input items [pos_bound[x], pos_bound[x + 1])
    uint32_t *cbase;                  // kMaxPasses * kChunks * kChunkRadix words (chunked sorts)
    uint32_t *chunk_ctr;              // kMaxPasses * kChunks tile counters, or NULL (no chunk fields)
    const uint32_t *mode;             // with chunked: nonzero if the probe chose per-chunk counts (NULL: chosen)
    uint32_t *user_k;
    uint32_t *user_v;
    uint32_t *t1_k;
    uint32_t *t1_v;
    uint32_t *t2_k;
    uint32_t *t2_v;
};

// ---- segmented sort (batched calls and the server)

constexpr int kSegBits = 8;
constexpr int kSegPasses = 4;
constexpr int kSegRadix = 1 << kSegBits;
constexpr int kSegTile = 1024 * 16;  // items per tile of the server's passes (batched calls: tuned)
constexpr int kSegMaxClasses = 4;    // whole-in-LDS size classes at most
constexpr uint32_t kSegLdsMax = 1024 * 16;  // largest segment one block sorts in LDS
constexpr uint32_t kLdsBytesPerCu = 160 * 1024;  // LDS of one gfx950 CU
constexpr int kSegLarge = kSegMaxClasses;   // list index of the tiled segments
constexpr uint32_t kSegErrBounds = 2u;  // a segment reached past the workspace

// Size limits of the whole-in-LDS classes of a call: class c takes the
// segments of more than max_n[c - 1] and at most max_n[c] items (increasing,
// at most kSegLdsMax); larger segments are tiled.
struct SegClassLimits {
    uint32_t count;
    uint32_t max_n[kSegMaxClasses];
};

// One segment.  The sorted result ends in k/v (the segment's own arrays);
// tk/tv are temporaries of n elements.  v and tv are NULL for keys only.
struct SegDesc {
    uint32_t *k, *v;
    uint32_t *tk, *tv;
    uint32_t n;
    uint32_t pass;  // pass to run when the launch does not fix one
    uint32_t row;   // row of the per-segment histogram and base tables
    uint32_t pad;
};

// Device-side counters of a segmented sort.
struct SegHeader {
    uint32_t count[kSegMaxClasses + 1];  // list lengths: whole-in-LDS classes, tiled
    uint32_t total_tiles;                // tiles of the tiled list
    uint32_t error;
    // XCD chunks of the tile list, cut at segment ends: chunk x holds tiles
    // [chunk_start[x], chunk_start[x + 1]); kChunks tile counters per launch
    uint32_t chunk_start[kChunks + 1];
    uint32_t chunk_ctr[kSegPasses + 1][kChunks];
};
static_assert(sizeof(SegHeader) <= 256, "two headers share 512 bytes in the server's metadata");

}  // namespace rt
