// rt_batched.hip -- host side of the batched segmented sort: workspace
// layout, launch sequence and the C ABI entry points.  The segment offsets
// stay on the device: descriptors, size classes and tile maps are all built
// by kernels, so a call is a fixed sequence of launches (no host sync) that
// a caller with its own workspace can capture into a HIP graph.
#include <cstring>
#include <mutex>

#include "rt_common.h"
#include "rt_seg_kernels.h"

namespace rt {

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

SegClassLimits SegClassTable::limits() const {
    SegClassLimits l{};
    l.count = count;
    for (uint32_t c = 0; c < count; ++c) l.max_n[c] = cls[c].max_n;
    return l;
}

bool seg_small_shape_supported(int block, int ipt, int bits) {
#define RT_SEG_SHAPE_CASE(BLK, I, B) \
    if (block == BLK && ipt == I && bits == B) return true;
    RT_FOR_EACH_SEG_SMALL_SHAPE(RT_SEG_SHAPE_CASE)
#undef RT_SEG_SHAPE_CASE
    return false;
}

bool seg_tile_shape_supported(int block, int ipt) {
#define RT_SEG_TILE_CASE(BLK, I) \
    if (block == BLK && ipt == I) return true;
    RT_FOR_EACH_SEG_TILE_SHAPE(RT_SEG_TILE_CASE)
#undef RT_SEG_TILE_CASE
    return false;
}

void launch_seg_small(const SegClass &c, bool vals, uint32_t max_listed, hipStream_t stream, const SegDesc *descs,
                      const uint32_t *list, const SegHeader *h, int which, int key_bits, int to_temp) {
    // enough blocks to fill the CUs: more per CU for smaller shapes, as many
    // as the LDS holds (stage, per-wave counters and scratch rows)
    const uint32_t cus = static_cast<uint32_t>(device_cu_count());
    const uint32_t lds = static_cast<uint32_t>(c.block * c.ipt) * (vals ? 8u : 4u) +
                         static_cast<uint32_t>(c.block / 64) * ((1u << c.bits) + 64u) * 4u + 64u;
    const uint32_t per_cu = std::max<uint32_t>(
        {1u, kSegLdsMax / static_cast<uint32_t>(c.block * c.ipt), kLdsBytesPerCu / lds});
    const uint32_t grid = std::max<uint32_t>(1u, std::min<uint32_t>(max_listed, cus * per_cu));
#define RT_SEG_SHAPE_LAUNCH(BLK, I, B)                                                                           \
    if (c.block == BLK && c.ipt == I && c.bits == B) {                                                           \
        if (vals)                                                                                                \
            hipLaunchKernelGGL((k_seg_small<BLK, I, true, B>), dim3(grid), dim3(BLK), 0, stream, descs, list, h, \
                               which, key_bits, to_temp);                                                        \
        else                                                                                                     \
            hipLaunchKernelGGL((k_seg_small<BLK, I, false, B>), dim3(grid), dim3(BLK), 0, stream, descs, list,   \
                               h, which, key_bits, to_temp);                                                     \
        return;                                                                                                  \
    }
    RT_FOR_EACH_SEG_SMALL_SHAPE(RT_SEG_SHAPE_LAUNCH)
#undef RT_SEG_SHAPE_LAUNCH
}

SegLayout make_seg_layout(uint32_t num_segments, size_t capacity, bool with_values, bool own_temps,
                          bool tiled_only, const SegClassTable *classes) {
    SegLayout L{};
    L.num_segments = num_segments;
    L.capacity = capacity;
    L.classes = classes ? *classes : seg_class_table();
    if (tiled_only) L.classes.count = 0;
    const size_t large_cap = std::min<size_t>(num_segments, capacity / (L.classes.lds_max() + 1));
    L.large_capacity = static_cast<uint32_t>(large_cap);
    L.tile = L.classes.tile();
    L.max_tiles = static_cast<uint32_t>((capacity + L.tile - 1) / L.tile + large_cap);
    L.wide_status = capacity >= (static_cast<size_t>(1) << 30);
    const size_t sw = L.wide_status ? 8 : 4;
    size_t off = 0;
    L.header = off;     off += align256(sizeof(SegHeader));
    L.descs = off;      off += align256(sizeof(SegDesc) * num_segments);
    L.lists = off;      off += align256(sizeof(uint32_t) * (kSegMaxClasses + 1) * static_cast<size_t>(num_segments));
    L.first_tile = off; off += align256(sizeof(uint32_t) * (large_cap + 1));
    L.tile_seg = off;   off += align256(sizeof(SegDesc) * L.max_tiles);
    L.hist = off;       off += align256(sizeof(uint32_t) * kSegPasses * kSegRadix * large_cap);
    L.base = off;       off += align256(sizeof(uint32_t) * kSegPasses * kSegRadix * large_cap);
    L.status_pass = static_cast<size_t>(L.max_tiles) * kSegRadix * sw;
    L.status = off;     off += align256(L.status_pass * kSegPasses);
    L.tk = L.tv = 0;
    if (own_temps) {
        L.tk = off;
        off += align256(sizeof(uint32_t) * capacity);
        if (with_values) { L.tv = off; off += align256(sizeof(uint32_t) * capacity); }
    }
    L.total = off;
    return L;
}

static uint32_t cap_grid(size_t want, uint32_t cap) {
    if (want < 1) want = 1;
    return static_cast<uint32_t>(want < cap ? want : cap);
}

// Per-segment histograms and prefix sums, whole-in-LDS segments, and passes
// 0..passes-1 (on digits digit0..digit0 + passes - 1) over the tiled
// segments.  The lists and the tiled list's counter are already on the
// device.  to_temp: the result is wanted in the temporaries (odd pass
// counts), where the tiled passes leave it.  persistent: the passes run one
// block per CU, each claiming tiles until none is left.
template <bool VALS, typename S>
static void launch_seg_sort_body(const SegPointers &P, const SegLayout &L, uint32_t list_stride, int passes,
                                 int to_temp, uint32_t nchunks, uint32_t digit0, bool persistent,
                                 hipStream_t stream) {
    const uint32_t cus = static_cast<uint32_t>(device_cu_count());
    uint32_t *large_list = P.lists + static_cast<size_t>(kSegLarge) * list_stride;
    hipLaunchKernelGGL(k_seg_tiles, dim3(1), dim3(1024), 0, stream, P.descs, large_list, P.first_tile, P.header,
                       L.large_capacity, L.max_tiles, L.tile);
    hipLaunchKernelGGL(k_seg_tilemap, dim3(cap_grid((L.max_tiles + 255) / 256, cus * 4)), dim3(256), 0, stream,
                       P.descs, large_list, P.first_tile, P.header, P.tile_seg, nchunks);
    prof_mark(stream, RT_KIND_SEGMENTED);
    // the histogram rows and lookback words this call uses start at zero
    hipLaunchKernelGGL(k_seg_clear, dim3(cus * 4), dim3(256), 0, stream, P.header, P.hist,
                       reinterpret_cast<uint32_t *>(P.status), L.status_pass / 4, L.wide_status ? 2u : 1u, passes);
    prof_mark(stream, RT_KIND_FILL);
    hipLaunchKernelGGL((k_seg_histogram<512, 16>), dim3(cap_grid(L.max_tiles, cus * 2)), dim3(512), 0, stream,
                       P.tile_seg, P.header, P.hist, L.tile,
                       ((1u << passes) - 1u) << digit0);
    prof_mark(stream, RT_KIND_HISTOGRAM);
    hipLaunchKernelGGL(k_seg_plan, dim3(cap_grid(L.large_capacity, cus * 4)), dim3(256), 0, stream, P.descs,
                       large_list, P.header, P.hist, P.base);
    prof_mark(stream, RT_KIND_PLAN);
    // whole-in-LDS classes
    for (uint32_t c = 0; c < L.classes.count; ++c)
        launch_seg_small(L.classes.cls[c], VALS, list_stride, stream, P.descs,
                         P.lists + static_cast<size_t>(c) * list_stride, P.header, static_cast<int>(c),
                         passes * kSegBits, to_temp);
    prof_mark(stream, RT_KIND_SEG_SMALL);
    for (int p = 0; p < passes; ++p) {
        S *status = reinterpret_cast<S *>(reinterpret_cast<char *>(P.status) + p * L.status_pass);
        uint32_t *ctr = P.header_words + offsetof(SegHeader, chunk_ctr) / 4 + p * kChunks;
        uint32_t *err = P.header_words + offsetof(SegHeader, error) / 4;
#define RT_SEG_TILE_LAUNCH(BLK, I)                                                                               \
    if (L.classes.tile_block == BLK && L.classes.tile_ipt == I) {                                                \
        if (persistent)                                                                                          \
            hipLaunchKernelGGL((k_seg_onesweep<BLK, I, VALS, S, true>), dim3(cap_grid(L.max_tiles, cus)),        \
                               dim3(BLK), 0, stream, P.tile_seg, P.header, p,                                    \
                               P.base, status, ctr, err, nchunks, digit0);                                       \
        else                                                                                                     \
            hipLaunchKernelGGL((k_seg_onesweep<BLK, I, VALS, S>), dim3(L.max_tiles), dim3(BLK), 0, stream,       \
                               P.tile_seg, P.header, p, P.base, status, ctr,                                     \
                               err, nchunks, digit0);                                                            \
    }
        RT_FOR_EACH_SEG_TILE_SHAPE(RT_SEG_TILE_LAUNCH)
#undef RT_SEG_TILE_LAUNCH
        prof_mark(stream, RT_KIND_PASS + p);
    }
}

SegPointers seg_pointers(char *ws, const SegLayout &L) {
    SegPointers P{};
    P.header = reinterpret_cast<SegHeader *>(ws + L.header);
    P.header_words = reinterpret_cast<uint32_t *>(ws + L.header);
    P.descs = reinterpret_cast<SegDesc *>(ws + L.descs);
    P.lists = reinterpret_cast<uint32_t *>(ws + L.lists);
    P.first_tile = reinterpret_cast<uint32_t *>(ws + L.first_tile);
    P.tile_seg = reinterpret_cast<SegDesc *>(ws + L.tile_seg);
    P.hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    P.base = reinterpret_cast<uint32_t *>(ws + L.base);
    P.status = ws + L.status;
    P.tk = reinterpret_cast<uint32_t *>(ws + L.tk);
    P.tv = L.tv ? reinterpret_cast<uint32_t *>(ws + L.tv) : nullptr;
    return P;
}

void launch_segments(uint32_t *keys, uint32_t *vals, uint32_t *tk, uint32_t *tv, const uint32_t *offsets,
                     uint32_t num_segments, const SegLayout &L, char *ws, int passes, int to_temp,
                     hipStream_t stream, uint32_t digit0, bool persistent) {
    const SegPointers P = seg_pointers(ws, L);
    const bool vals_on = vals != nullptr;
    hipLaunchKernelGGL(k_seg_reset, dim3(1), dim3(64), 0, stream, P.header);
    hipLaunchKernelGGL(k_seg_classify, dim3((num_segments + 255) / 256), dim3(256), 0, stream, offsets,
                       num_segments, keys, vals, tk, vals_on ? tv : nullptr, L.capacity, L.large_capacity,
                       to_temp, L.classes.limits(), P.descs, P.lists, P.header);
    // XCD chunks of the tile list pay off for long segments only: with a few
    // tiles per segment (many partial tiles, short lookback chains) one
    // chunk measured faster.  The segments' mean size bounds their tiles.
    const uint32_t nchunks = seg_chunk_count(L.capacity, num_segments, L.tile);
    if (L.wide_status) {
        if (vals_on) launch_seg_sort_body<true, uint64_t>(P, L, num_segments, passes, to_temp, nchunks, digit0, persistent, stream);
        else launch_seg_sort_body<false, uint64_t>(P, L, num_segments, passes, to_temp, nchunks, digit0, persistent, stream);
    } else {
        if (vals_on) launch_seg_sort_body<true, uint32_t>(P, L, num_segments, passes, to_temp, nchunks, digit0, persistent, stream);
        else launch_seg_sort_body<false, uint32_t>(P, L, num_segments, passes, to_temp, nchunks, digit0, persistent, stream);
    }
}

void launch_batched(uint32_t *keys, uint32_t *vals, const uint32_t *offsets, uint32_t num_segments,
                    const SegLayout &L, char *ws, hipStream_t stream) {
    const SegPointers P = seg_pointers(ws, L);
    prof_begin(stream);
    launch_segments(keys, vals, P.tk, vals ? P.tv : nullptr, offsets, num_segments, L, ws, kSegPasses, 0, stream);
}

}  // namespace rt

using namespace rt;

static rt_status check_batched(uint32_t *keys, uint32_t *vals, const uint32_t *seg_offsets, uint32_t num_segments,
                               size_t max_total, const char *what) {
    if (max_total >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "%s: max_total = %zu, the limit is 2^32 - 1", what, max_total);
    if (num_segments == 0 || max_total < 2) return RT_OK;
    if (seg_offsets == nullptr) return set_error(RT_ERR_INVALID_ARG, "%s: seg_offsets is NULL", what);
    if (keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "%s: keys is NULL", what);
    if ((reinterpret_cast<uintptr_t>(keys) | reinterpret_cast<uintptr_t>(vals) |
         reinterpret_cast<uintptr_t>(seg_offsets)) & 3u)
        return set_error(RT_ERR_INVALID_ARG, "%s: arrays must be 4-byte aligned", what);
    if (vals != nullptr && keys == vals) return set_error(RT_ERR_INVALID_ARG, "%s: keys and values alias", what);
    return RT_OK;
}

extern "C" size_t rt_batched_workspace_bytes(uint32_t num_segments, size_t max_total, int with_values) {
    if (num_segments == 0 || max_total < 2 || max_total >= (static_cast<size_t>(1) << 32)) return 0;
    return make_seg_layout(num_segments, max_total, with_values != 0, true).total;
}

extern "C" rt_status rt_sort_batched_ex(uint32_t *keys, uint32_t *vals, const uint32_t *seg_offsets,
                                        uint32_t num_segments, size_t max_total, uint32_t flags, void *workspace,
                                        size_t workspace_bytes, hipStream_t stream) {
    rt_status s = check_batched(keys, vals, seg_offsets, num_segments, max_total, "rt_sort_batched_ex");
    if (s != RT_OK || num_segments == 0 || max_total < 2) return s;
    if (flags & ~static_cast<uint32_t>(RT_FLAG_VALIDATE))
        return set_error(RT_ERR_INVALID_ARG, "rt_sort_batched_ex: unknown flags 0x%x", flags);
    const SegLayout L = make_seg_layout(num_segments, max_total, vals != nullptr, true);
    void *ws = workspace;
    if (ws != nullptr) {
        if (workspace_bytes < L.total)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort_batched_ex: workspace of %zu bytes, %zu needed",
                             workspace_bytes, L.total);
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort_batched_ex: workspace must be 256-byte aligned");
    } else {
        s = cached_workspace(L.total, stream, &ws);
        if (s != RT_OK) return s;
    }
    launch_batched(keys, vals, seg_offsets, num_segments, L, static_cast<char *>(ws), stream);
    s = finish_call(stream, "rt_sort_batched_ex");
    if (s != RT_OK) return s;
    if ((flags & RT_FLAG_VALIDATE) || debug_sync_enabled()) {
        SegHeader h;
        hipError_t e = hipMemcpyAsync(&h, static_cast<char *>(ws) + L.header, sizeof h, hipMemcpyDeviceToHost,
                                      stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "rt_sort_batched_ex: %s", hipGetErrorString(e));
        if (h.error & kSegErrBounds)
            return set_error(RT_ERR_INVALID_ARG,
                             "rt_sort_batched_ex: malformed offsets (decreasing, or past max_total); those "
                             "segments were left unsorted");
        if (h.error) return set_error(RT_ERR_HIP, "rt_sort_batched_ex: device error word 0x%x", h.error);
    }
    return RT_OK;
}

extern "C" rt_status rt_sort_pairs_batched(uint32_t *keys, uint32_t *vals, const uint32_t *seg_offsets,
                                           uint32_t num_segments, size_t max_total, hipStream_t stream) {
    return rt_sort_batched_ex(keys, vals, seg_offsets, num_segments, max_total, 0u, nullptr, 0, stream);
}
