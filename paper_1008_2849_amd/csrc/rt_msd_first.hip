// rt_msd_first.hip -- "reverse sorting" (Section 4, Algorithm 2) on one
// GPU: one counting-sort pass on the most significant 8-bit digit moves the
// caller's arrays into a temporary, partitioned into 256 MSD buckets; then
// every bucket is sorted on its own by LSD passes over digits 0, 1 and 2,
// the last of which writes the caller's arrays.
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
#include "rt_common.h"
#include "rt_kernels.h"

namespace rt {

namespace {
constexpr uint32_t kMsdShift = 24;
constexpr uint32_t kMsdWidth = 8;
constexpr uint32_t kMsdBuckets = 1u << kMsdWidth;
constexpr int kLocalPasses = 3;

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct MsdLayout {
    Resolved r;       // the partition pass
    Layout part;      // its histogram, plan and lookback words (at offset 0)
    size_t tk, tv;    // the partitioned copy
    size_t seg;       // the segmented sort's tables
    SegLayout local;
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
    M.seg = off;
    M.local = make_seg_layout(kMsdBuckets, n, with_values, false);
    M.total = off + M.local.total;
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
    if (flags & ~static_cast<uint32_t>(RT_FLAG_VALIDATE))
        return set_error(RT_ERR_INVALID_ARG, "%s: unknown flags 0x%x", what, flags);
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
    // local LSD over digits 0..2 of each bucket: temporary -> caller's arrays
    const uint32_t *bucket_offsets = reinterpret_cast<const uint32_t *>(w + M.part.base);
    launch_segments(tk, tv, keys, vals, bucket_offsets, kMsdBuckets, M.local, w + M.seg, kLocalPasses, 1, stream);
    rt_status s = finish_call(stream, what);
    if (s != RT_OK) return s;
    if ((flags & RT_FLAG_VALIDATE) || debug_sync_enabled()) {
        uint32_t part_err = 0;
        SegHeader h;
        hipError_t e = hipMemcpyAsync(&part_err, w + M.part.ctr + sizeof(uint32_t) * kMaxPasses, sizeof part_err,
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&h, w + M.seg + M.local.header, sizeof h, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
        if (part_err || h.error)
            return set_error(RT_ERR_HIP, "%s: device error words 0x%x (partition), 0x%x (local passes)", what,
                             part_err, h.error);
    }
    return RT_OK;
}
