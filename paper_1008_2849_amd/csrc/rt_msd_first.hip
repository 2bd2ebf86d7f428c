// rt_msd_first.hip -- "reverse sorting" (Section 4, Algorithm 2) on one
// GPU: one counting-sort pass on the most significant 8-bit digit moves the
// caller's arrays into a temporary, partitioned into 256 MSD buckets; then
// every bucket is sorted on its own by LSD passes over digits 0, 1 and 2,
// the last of which writes the caller's arrays.
//
// The paper partitions until a bucket fits the cache and sorts it there.
// On this GPU the fast memory a bucket can be sorted in is one block's LDS
// (16K items), so large inputs take a second MSD level: a segmented pass on
// digit 2 inside the buckets (their digit-2 counts, one read, give 65536
// sub-bucket bounds), then digits 0 and 1 of each sub-bucket, whole in LDS
// when it fits, else by two tiled passes.  Three passes over HBM instead of
// four, the last of them with two digits' work in LDS.
//
// Algorithm 2's pieces map as follows.  The MSD histogram and its exclusive
// prefix sum (bucketSizes, outputIndices) are the upfront histogram and plan
// kernels of the single-array sort restricted to digit 3; the partition is
// one onesweep pass.  The plan kernel leaves outputIndices in the base table
// with n past the last bin, which is exactly the segment offset array of the
// segmented sort, so the buckets become segments without a host round trip.
// The local passes are the segmented sort's: buckets of at most 16K items
// are sorted whole in LDS, larger ones by three onesweep passes whose
// lookback chains end at the bucket's first tile.  The local histograms of
// digits 0..2 are taken in one read of each bucket before its first local
// pass (Algorithm 2 has no need for the first two: its buckets grow in
// virtual memory).
#include <algorithm>

#include "rt_common.h"
#include "rt_seg_kernels.h"

namespace rt {

namespace {
constexpr uint32_t kMsdShift = 24;
constexpr uint32_t kMsdWidth = 8;
constexpr uint32_t kMsdBuckets = 1u << kMsdWidth;
constexpr int kLocalPasses = 3;
constexpr uint32_t kSubBuckets = kMsdBuckets << 8;  // second level: digit 2 inside each bucket
// Two levels by default from this size (sub-buckets of about 1024 items and
// up, with the classes of leaf_classes): measured faster than one level at
// 2^26, 2^27 and 2^28 items.
constexpr size_t kTwoLevelMinItems = static_cast<size_t>(1) << 26;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Size classes of the sub-buckets.  Uniform keys give sub-buckets of about
// m = n / 65536 items, within a few sqrt(m).  The first class sits about
// four standard deviations above m, so one launch of blocks hardly larger
// than the sub-buckets takes nearly all of them: 256 x 17 (4352 items) for
// m = 4096 (2^28 items), 256 x 9 (2304) for m = 2048, 128 x 9 (1152) for
// m = 1024; the rare larger ones go to the next classes.  Smaller m keeps
// the tuned classes.
SegClassTable leaf_classes(size_t n) {
    SegClassTable t = seg_class_table();
    const size_t m = n / kSubBuckets;
    if (m < 768) return t;
    t.count = 4;
    if (m >= 3072) {
        t.count = 3;
        t.cls[0] = SegClass{4352, 256, 17, 8};
        t.cls[1] = SegClass{8192, 512, 16, 8};
        t.cls[2] = SegClass{16384, 1024, 16, 8};
    } else if (m >= 1536) {
        t.cls[0] = SegClass{2304, 256, 9, 8};
        t.cls[1] = SegClass{4352, 256, 17, 8};
        t.cls[2] = SegClass{8192, 512, 16, 8};
        t.cls[3] = SegClass{16384, 1024, 16, 8};
    } else {
        t.cls[0] = SegClass{1152, 128, 9, 8};
        t.cls[1] = SegClass{2304, 256, 9, 8};
        t.cls[2] = SegClass{4352, 256, 17, 8};
        t.cls[3] = SegClass{16384, 1024, 16, 8};
    }
    return t;
}

struct MsdLayout {
    Resolved r;       // the partition pass
    Layout part;      // its histogram, plan and lookback words (at offset 0)
    size_t tk, tv;    // the partitioned copy
    size_t sub;       // two levels: sub-bucket offsets (kSubBuckets + 1), then the first level's error word
    size_t seg;       // the segmented sorts' tables (one call at a time)
    SegLayout local;  // one level: digits 0..2 of every bucket
    SegLayout level2; // two levels: digit 2 of every bucket (tiled only)
    SegLayout leaf;   // two levels: digits 0..1 of every sub-bucket
    size_t total;
};

MsdLayout make_msd_layout(size_t n, bool with_values) {
    MsdLayout M{};
    rt_config t;
    tuned_config(n, with_values, &t);
    Resolved &r = M.r;
    r.num_passes = 1;
    r.shift[0] = kMsdShift;
    r.width[0] = kMsdWidth;
    r.block = static_cast<int>(t.block_threads);
    r.ipt = static_cast<int>(t.items_per_thread);
    if (!shape_supported(8, r.block, r.ipt)) {
        r.block = 1024;
        r.ipt = 16;
    }
    r.flags = RT_FLAG_NO_SKIP | (t.flags & RT_FLAG_NT_STORES);
    r.with_values = with_values;
    // the partition pass runs in XCD chunks by position when the probe agrees
    r.chunked = n >= kChunkMinItems;
    r.probe = r.chunked;
    M.part = make_layout(n, r, true);
    size_t off = align256(M.part.total);
    M.tk = off;
    off += align256(n * sizeof(uint32_t));
    M.tv = 0;
    if (with_values) {
        M.tv = off;
        off += align256(n * sizeof(uint32_t));
    }
    M.sub = off;
    off += align256(sizeof(uint32_t) * (kSubBuckets + 2));
    M.seg = off;
    M.local = make_seg_layout(kMsdBuckets, n, with_values, false);
    M.level2 = make_seg_layout(kMsdBuckets, n, with_values, false, true);
    const SegClassTable leaf = leaf_classes(n);
    M.leaf = make_seg_layout(kSubBuckets, n, with_values, false, false, &leaf);
    M.total = off + std::max(M.local.total, std::max(M.level2.total, M.leaf.total));
    return M;
}
}  // namespace

}  // namespace rt

using namespace rt;

extern "C" size_t rt_msd_first_workspace_bytes(size_t n, int with_values) {
    if (n < 2 || n >= (static_cast<size_t>(1) << 32)) return 0;
    return make_msd_layout(n, with_values != 0).total;
}

extern "C" rt_status rt_sort_msd_first(uint32_t *keys, uint32_t *vals, size_t n, uint32_t flags, void *workspace,
                                       size_t workspace_bytes, hipStream_t stream) {
    const char *what = "rt_sort_msd_first";
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "%s: n = %zu, the limit is 2^32 - 1", what, n);
    if (flags & ~static_cast<uint32_t>(RT_FLAG_VALIDATE | RT_FLAG_MSD_ONE_LEVEL | RT_FLAG_MSD_TWO_LEVELS))
        return set_error(RT_ERR_INVALID_ARG, "%s: unknown flags 0x%x", what, flags);
    if ((flags & RT_FLAG_MSD_ONE_LEVEL) && (flags & RT_FLAG_MSD_TWO_LEVELS))
        return set_error(RT_ERR_INVALID_ARG, "%s: RT_FLAG_MSD_ONE_LEVEL and RT_FLAG_MSD_TWO_LEVELS exclude each other",
                         what);
    if (n < 2) return RT_OK;
    if (keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "%s: keys is NULL with n = %zu", what, n);
    if ((reinterpret_cast<uintptr_t>(keys) | reinterpret_cast<uintptr_t>(vals)) & 3u)
        return set_error(RT_ERR_INVALID_ARG, "%s: arrays must be 4-byte aligned", what);
    if (vals != nullptr) {
        const uintptr_t k0 = reinterpret_cast<uintptr_t>(keys), v0 = reinterpret_cast<uintptr_t>(vals);
        const uintptr_t bytes = n * sizeof(uint32_t);
        if (k0 < v0 + bytes && v0 < k0 + bytes)
            return set_error(RT_ERR_INVALID_ARG, "%s: keys and values overlap", what);
    }
    const MsdLayout M = make_msd_layout(n, vals != nullptr);
    void *ws = workspace;
    if (ws != nullptr) {
        if (workspace_bytes < M.total)
            return set_error(RT_ERR_INVALID_ARG, "%s: workspace of %zu bytes, %zu needed", what, workspace_bytes,
                             M.total);
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return set_error(RT_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", what);
    } else {
        rt_status s = cached_workspace(M.total, stream, &ws);
        if (s != RT_OK) return s;
    }
    char *w = static_cast<char *>(ws);
    uint32_t *tk = reinterpret_cast<uint32_t *>(w + M.tk);
    uint32_t *tv = vals ? reinterpret_cast<uint32_t *>(w + M.tv) : nullptr;
    // partition: caller's arrays -> temporary, by the MSD
    launch_sort(keys, vals, static_cast<uint32_t>(n), M.r, M.part, w, true, tk, tv, stream, RT_KIND_MSD_PASS);
    const uint32_t *bucket_offsets = reinterpret_cast<const uint32_t *>(w + M.part.base);
    const bool two = (flags & RT_FLAG_MSD_TWO_LEVELS) || (!(flags & RT_FLAG_MSD_ONE_LEVEL) && n >= kTwoLevelMinItems);
    uint32_t *sub = reinterpret_cast<uint32_t *>(w + M.sub);
    if (two) {
        // digit 2 inside every bucket: temporary -> caller's arrays
        launch_segments(tk, tv, keys, vals, bucket_offsets, kMsdBuckets, M.level2, w + M.seg, 1, 1, stream, 2);
        const SegPointers P = seg_pointers(w + M.seg, M.level2);
        hipLaunchKernelGGL(k_msd_subbuckets, dim3(kMsdBuckets), dim3(256), 0, stream, bucket_offsets, P.descs, P.hist,
                           2u, kMsdBuckets, sub, P.header, sub + kSubBuckets + 1);
        prof_mark(stream, RT_KIND_PLAN);
        // digits 0 and 1 of every sub-bucket, in the caller's arrays
        launch_segments(keys, vals, tk, tv, sub, kSubBuckets, M.leaf, w + M.seg, 2, 0, stream, 0, true);
    } else {
        // local LSD over digits 0..2 of each bucket: temporary -> caller's arrays
        launch_segments(tk, tv, keys, vals, bucket_offsets, kMsdBuckets, M.local, w + M.seg, kLocalPasses, 1, stream);
    }
    rt_status s = finish_call(stream, what);
    if (s != RT_OK) return s;
    if ((flags & RT_FLAG_VALIDATE) || debug_sync_enabled()) {
        uint32_t part_err = 0, level2_err = 0;
        SegHeader h;
        hipError_t e = hipMemcpyAsync(&part_err, w + M.part.ctr + sizeof(uint32_t) * kMaxPasses, sizeof part_err,
                                      hipMemcpyDeviceToHost, stream);
        // every segmented layout starts with its header, at M.seg
        if (e == hipSuccess) e = hipMemcpyAsync(&h, w + M.seg, sizeof h, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess && two)
            e = hipMemcpyAsync(&level2_err, sub + kSubBuckets + 1, sizeof level2_err, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
        if (part_err || level2_err || h.error)
            return set_error(RT_ERR_HIP, "%s: device error words 0x%x (partition), 0x%x (second level), 0x%x (local passes)",
                             what, part_err, level2_err, h.error);
    }
    return RT_OK;
}
