// rt_sort.hip -- host side of the single-array sort: argument checks, tuned
// configuration, workspace layout and cache, kernel launch sequence, and the
// C ABI entry points declared in include/rtsort.h.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <map>
#include <vector>
#include <mutex>
#include <string>
#include <utility>

#include "rt_common.h"
#include "rt_kernels.h"

namespace rt {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string t_last_error;

rt_status set_error(rt_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return s;
}

const char *last_error() { return t_last_error.c_str(); }

bool debug_sync_enabled() {
    static const bool on = [] {
        const char *e = getenv("RT_DEBUG_SYNC");
        return e != nullptr && atoi(e) != 0;
    }();
    return on;
}

rt_status finish_call(hipStream_t stream, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    if (debug_sync_enabled()) {
        e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    }
    return RT_OK;
}

int device_cu_count() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    cache[dev] = cus;
    return cus;
}

// ---------------------------------------------------------------------------
// configuration
// ---------------------------------------------------------------------------

bool shape_supported(int bits_class, int block, int ipt) {
#define RT_SHAPE_CASE(B, BLK, I) \
    if (bits_class == B && block == BLK && ipt == I) return true;
    RT_FOR_EACH_SHAPE(RT_SHAPE_CASE)
#undef RT_SHAPE_CASE
    return false;
}

static int bits_class_of(uint32_t width) { return width <= 8 ? 8 : 11; }

rt_status resolve_config(const rt_config *cfg, size_t n, int with_values, Resolved *out) {
    rt_config c;
    if (cfg == nullptr || cfg->num_passes == 0) {
        tuned_config(n, with_values, &c);
        if (cfg != nullptr) {  // keep explicit block / ipt / flags over the tuned widths
            if (cfg->block_threads) c.block_threads = cfg->block_threads;
            if (cfg->items_per_thread) c.items_per_thread = cfg->items_per_thread;
            c.flags |= cfg->flags;
        }
    } else {
        c = *cfg;
        rt_config t;
        tuned_config(n, with_values, &t);
        if (c.block_threads == 0) c.block_threads = t.block_threads;
        if (c.items_per_thread == 0) c.items_per_thread = t.items_per_thread;
    }
    if (c.num_passes < 1 || c.num_passes > kMaxPasses)
        return set_error(RT_ERR_INVALID_ARG, "num_passes %u outside 1..%d", c.num_passes, kMaxPasses);
    uint32_t total = 0;
    Resolved r{};
    r.num_passes = c.num_passes;
    for (uint32_t p = 0; p < c.num_passes; ++p) {
        const uint32_t w = c.digit_bits[p];
        if (w < 1 || w > static_cast<uint32_t>(kMaxBits))
            return set_error(RT_ERR_INVALID_ARG, "digit_bits[%u] = %u outside 1..%d", p, w, kMaxBits);
        r.shift[p] = total;
        r.width[p] = w;
        total += w;
    }
    if (total != 32) return set_error(RT_ERR_INVALID_ARG, "digit widths sum to %u, not 32", total);
    r.block = static_cast<int>(c.block_threads);
    r.ipt = static_cast<int>(c.items_per_thread);
    const bool explicit_shape = cfg != nullptr && cfg->block_threads != 0 && cfg->items_per_thread != 0;
    if (!explicit_shape) {
        // the tuned tile may be too large for wider digits: use the widest
        // shape every digit class has
        bool ok = true;
        for (uint32_t p = 0; p < r.num_passes; ++p)
            ok = ok && shape_supported(bits_class_of(r.width[p]), r.block, r.ipt);
        if (!ok) {
            r.block = 512;
            r.ipt = 16;
        }
    }
    for (uint32_t p = 0; p < r.num_passes; ++p)
        if (!shape_supported(bits_class_of(r.width[p]), r.block, r.ipt))
            return set_error(RT_ERR_UNSUPPORTED, "no kernel for %d-bit digits with %d threads x %d items",
                             bits_class_of(r.width[p]), r.block, r.ipt);
    r.flags = c.flags;
    r.with_values = with_values != 0;
    if (r.flags & ~static_cast<uint32_t>(RT_FLAG_NO_SKIP | RT_FLAG_NT_STORES | RT_FLAG_DIRECT_SCATTER |
                                         RT_FLAG_ONE_CHAIN | RT_FLAG_CHUNKS | RT_FLAG_VALIDATE |
                                         RT_FLAG_FUSED_HISTOGRAM))
        return set_error(RT_ERR_INVALID_ARG, "unknown flags 0x%x", r.flags);
    r.fused = (r.flags & RT_FLAG_FUSED_HISTOGRAM) != 0;
    if (r.fused) {
        if (r.flags & RT_FLAG_CHUNKS)
            return set_error(RT_ERR_UNSUPPORTED, "RT_FLAG_FUSED_HISTOGRAM runs on one chain: not with RT_FLAG_CHUNKS");
        if (r.flags & (RT_FLAG_DIRECT_SCATTER | RT_FLAG_NT_STORES))
            return set_error(RT_ERR_UNSUPPORTED,
                             "RT_FLAG_FUSED_HISTOGRAM is built for the staged pass with plain stores only");
        for (uint32_t p = 0; p < r.num_passes; ++p)
            if (r.width[p] > 8)
                return set_error(RT_ERR_UNSUPPORTED, "RT_FLAG_FUSED_HISTOGRAM needs digits of at most 8 bits");
        // the later histograms do not exist when the buffers are planned
        r.flags |= RT_FLAG_NO_SKIP | RT_FLAG_ONE_CHAIN;
    }
    if ((r.flags & RT_FLAG_ONE_CHAIN) && (r.flags & RT_FLAG_CHUNKS))
        return set_error(RT_ERR_INVALID_ARG, "RT_FLAG_ONE_CHAIN and RT_FLAG_CHUNKS exclude each other");
    if (r.block == 512 && r.ipt == 32 &&
        (r.flags & (RT_FLAG_NT_STORES | RT_FLAG_DIRECT_SCATTER | RT_FLAG_FUSED_HISTOGRAM)))
        return set_error(RT_ERR_UNSUPPORTED, "512 x 32 tiles are built for the staged pass with plain stores only");
    // per-chunk counts need digits of at most 8 bits (kChunkRadix); below
    // kChunkMinItems the sample would cost more than chunks can save
    const bool forced = (r.flags & RT_FLAG_CHUNKS) != 0;
    r.chunked = !(r.flags & RT_FLAG_ONE_CHAIN) && (forced || n >= kChunkMinItems);
    for (uint32_t p = 0; p < r.num_passes; ++p) r.chunked = r.chunked && r.width[p] <= 8;
    r.probe = r.chunked && !forced;
    if ((r.flags & RT_FLAG_DIRECT_SCATTER) && (r.flags & RT_FLAG_NT_STORES))
        return set_error(RT_ERR_UNSUPPORTED, "RT_FLAG_DIRECT_SCATTER with RT_FLAG_NT_STORES is not built");
    *out = r;
    return RT_OK;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

Layout make_layout(size_t n, const Resolved &r, bool direct) {
    Layout L{};
    const size_t tile = static_cast<size_t>(r.block) * r.ipt;
    const size_t tiles = (n + tile - 1) / tile;
    L.tiles = static_cast<uint32_t>(tiles);
    L.grid_tiles = static_cast<uint32_t>(tiles + (r.chunked ? kChunks - 1 : 0));
    L.wide_status = n >= (static_cast<size_t>(1) << 30);
    const size_t sw = L.wide_status ? 8 : 4;
    // the histograms and the lookback words are adjacent: one fill clears
    // both.  Per-chunk histograms (kMaxPasses * kChunks * kChunkRadix words)
    // fit the plain ones' space.
    static_assert(kChunks * kChunkRadix <= kMaxRadix, "per-chunk histograms must fit the plain ones' space");
    size_t off = 0;
    L.hist = off;    off += align256(sizeof(uint32_t) * kMaxPasses * kMaxRadix);
    L.status = off;
    for (uint32_t p = 0; p < r.num_passes; ++p) {
        L.status_pass[p] = off - L.status;
        off += L.grid_tiles * (static_cast<size_t>(1) << (r.width[p] <= 8 ? 8 : 11)) * sw;
    }
    off = align256(off);
    L.status_bytes = off - L.status;
    // tile counters of the passes, the error word, kChunks tile counters per
    // pass, the probe's choice
    L.ctr = off;     off += align256(sizeof(uint32_t) * (kMaxPasses + 2 + kMaxPasses * kChunks));
    L.base = off;    off += align256(sizeof(uint32_t) * kMaxPasses * kMaxRadix);
    L.cbase = off;   off += align256(sizeof(uint32_t) * kMaxPasses * kChunks * kChunkRadix);
    L.plan = off;    off += align256(sizeof(SortPlan));
    L.t1k = L.t1v = L.t2k = L.t2v = 0;
    if (!direct) {
        // A second temporary is needed whenever the executed pass count can
        // be odd and at least three: the pass count is odd, or passes may be
        // skipped at run time.
        const bool need_t2 = (r.num_passes & 1u) || !(r.flags & RT_FLAG_NO_SKIP);
        const size_t arr = align256(n * sizeof(uint32_t));
        L.t1k = off; off += arr;
        if (r.with_values) { L.t1v = off; off += arr; }
        if (need_t2) {
            L.t2k = off; off += arr;
            if (r.with_values) { L.t2v = off; off += arr; }
        }
    }
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// workspace cache: one growable buffer per (device, stream)
// ---------------------------------------------------------------------------

namespace {
struct CacheEntry {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, CacheEntry> g_ws;
}  // namespace

rt_status cached_workspace(size_t bytes, hipStream_t stream, void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    CacheEntry &c = g_ws[{dev, stream}];
    if (c.bytes < bytes) {
        // Stream-ordered growth: the old buffer is freed, and the new one
        // allocated, in the stream's order, behind the work that may still
        // use the old one, so the host never waits.
        if (c.ptr != nullptr) {
            e = hipFreeAsync(c.ptr, stream);
            if (e != hipSuccess) return set_error(RT_ERR_HIP, "hipFreeAsync: %s", hipGetErrorString(e));
            c.ptr = nullptr;
            c.bytes = 0;
        }
        void *p = nullptr;
        e = hipMallocAsync(&p, bytes, stream);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(RT_ERR_OUT_OF_MEMORY, "hipMallocAsync(%zu) for the workspace: %s", bytes,
                             hipGetErrorString(e));
        }
        c.ptr = p;
        c.bytes = bytes;
    }
    *out = c.ptr;
    return RT_OK;
}

rt_status read_device_word(const void *word, hipStream_t stream, uint32_t *out, const char *what) {
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(out, word, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return RT_OK;
}

// ---------------------------------------------------------------------------
// kernel timing marks
// ---------------------------------------------------------------------------

namespace {
struct Mark {
    hipEvent_t ev;
    hipStream_t stream;
    uint32_t kind;  // 0: start of a call
};
std::atomic<bool> g_prof_on{false};
std::mutex g_prof_mu;
std::vector<hipEvent_t> g_prof_events;
std::vector<Mark> g_prof_marks;
}  // namespace

static void prof_record(hipStream_t stream, uint32_t kind) {
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    const size_t i = g_prof_marks.size();
    if (i >= g_prof_events.size()) return;
    if (hipEventRecord(g_prof_events[i], stream) != hipSuccess) return;
    g_prof_marks.push_back(Mark{g_prof_events[i], stream, kind});
}

void prof_begin(hipStream_t stream) { prof_record(stream, 0u); }
void prof_mark(hipStream_t stream, uint32_t kind) { prof_record(stream, kind); }

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------

// fused_hist (RT_FLAG_FUSED_HISTOGRAM, not for a sort's last pass): the
// pass also counts the next pass's digit into that pass's row of it.
template <int BITS, int BLOCK, int IPT>
static void launch_pass_shape(const Layout &L, bool vals, uint32_t flags, hipStream_t stream, const SortPlan *plan,
                              int pass, uint32_t n, void *status, uint32_t *ctr, uint32_t kind,
                              uint32_t *fused_hist) {
    const dim3 grid(L.grid_tiles), block(BLOCK);
    uint32_t *err = ctr + kMaxPasses;
    uint32_t *chunk_ctr = ctr + kMaxPasses + 1 + pass * kChunks;
    const bool nt = (flags & RT_FLAG_NT_STORES) != 0;
    const bool stage = (flags & RT_FLAG_DIRECT_SCATTER) == 0;
#define RT_OS(V, NTV, S, STG, FU)                                                                                \
    hipLaunchKernelGGL((k_onesweep<BITS, BLOCK, IPT, V, NTV, S, STG, FU>), grid, block, 0, stream, plan, pass, n, \
                       static_cast<S *>(status), chunk_ctr, err, fused_hist)
    if constexpr (BLOCK == 512 && IPT == 32) {  // resolve_config: the plain staged pass only
        if (L.wide_status) { if (vals) RT_OS(true, false, uint64_t, true, false); else RT_OS(false, false, uint64_t, true, false); }
        else               { if (vals) RT_OS(true, false, uint32_t, true, false); else RT_OS(false, false, uint32_t, true, false); }
    } else if (fused_hist != nullptr) {  // resolve_config: staged, plain stores, digits of at most 8 bits
        if constexpr (BITS == 8) {
            if (L.wide_status) { if (vals) RT_OS(true, false, uint64_t, true, true); else RT_OS(false, false, uint64_t, true, true); }
            else               { if (vals) RT_OS(true, false, uint32_t, true, true); else RT_OS(false, false, uint32_t, true, true); }
        }
    } else if (!stage) {  // resolve_config rules out the non-temporal form here
        if (L.wide_status) { if (vals) RT_OS(true, false, uint64_t, false, false); else RT_OS(false, false, uint64_t, false, false); }
        else               { if (vals) RT_OS(true, false, uint32_t, false, false); else RT_OS(false, false, uint32_t, false, false); }
    } else if (L.wide_status) {
        if (vals) { if (nt) RT_OS(true, true, uint64_t, true, false); else RT_OS(true, false, uint64_t, true, false); }
        else      { if (nt) RT_OS(false, true, uint64_t, true, false); else RT_OS(false, false, uint64_t, true, false); }
    } else {
        if (vals) { if (nt) RT_OS(true, true, uint32_t, true, false); else RT_OS(true, false, uint32_t, true, false); }
        else      { if (nt) RT_OS(false, true, uint32_t, true, false); else RT_OS(false, false, uint32_t, true, false); }
    }
#undef RT_OS
    prof_mark(stream, kind);
}

static void launch_pass(int bits_class, int block, int ipt, const Layout &L, bool vals, uint32_t flags,
                        hipStream_t stream, const SortPlan *plan, int pass, uint32_t n, void *status,
                        uint32_t *ctr, uint32_t kind, uint32_t *fused_hist) {
#define RT_SHAPE_LAUNCH(B, BLK, I)                                                                           \
    if (bits_class == B && block == BLK && ipt == I) {                                                       \
        launch_pass_shape<B, BLK, I>(L, vals, flags, stream, plan, pass, n, status, ctr, kind, fused_hist); \
        return;                                                                                              \
    }
    RT_FOR_EACH_SHAPE(RT_SHAPE_LAUNCH)
#undef RT_SHAPE_LAUNCH
}

// Input items of pass 0's chunk x: [bound[x], bound[x + 1]), whole tiles,
// kChunks nearly equal shares of the tile grid.
void pos_bounds(size_t n, const Resolved &r, uint32_t bound[kChunks + 1]) {
    const uint64_t tile = static_cast<uint64_t>(r.block) * r.ipt;
    const uint64_t tiles = (n + tile - 1) / tile;
    for (int x = 0; x <= kChunks; ++x) bound[x] = static_cast<uint32_t>(std::min<uint64_t>(n, x * tiles / kChunks * tile));
    bound[kChunks] = static_cast<uint32_t>(n);
}

// chunked: per-chunk counts (see k_histogram), for sorts with r.chunked.
HistArgs hist_args(const Resolved &r, size_t n, bool chunked) {
    HistArgs ha{};
    ha.num_passes = r.num_passes;
    uint32_t off = 0;
    for (uint32_t p = 0; p < r.num_passes; ++p) {
        ha.shift[p] = r.shift[p];
        ha.mask[p] = (1u << r.width[p]) - 1u;
        ha.cshift[p] = r.width[p] > 3 ? r.width[p] - 3 : 0;
        ha.lds_offset[p] = off;
        off += (chunked ? kChunks : 1) << r.width[p];
    }
    ha.total_bins = off;
    if (chunked) pos_bounds(n, r, ha.pos_bound);
    return ha;
}

static uint32_t grid_for(size_t items, size_t per_block, uint32_t cap) {
    size_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<uint32_t>(g);
}

// LDS copies per block for a counter set of `bins` words: as many as fit
// in 64 KiB (padded rows), at most 16.
static int hist_copies(uint32_t bins) {
    int c = 16;
    while (c > 1 && static_cast<size_t>(c) * (bins + 1) * sizeof(uint32_t) > 72 * 1024) c /= 2;
    return c;
}

template <int C, bool CHUNKED>
static void launch_histogram_copies(const uint32_t *keys, uint32_t n, const HistArgs &ha, uint32_t *hist,
                                    hipStream_t stream) {
    constexpr int kBlock = 512;
    const size_t lds = static_cast<size_t>(C) * (ha.total_bins + 1) * sizeof(uint32_t);
    static std::once_flag once;  // dynamic LDS above 64 KiB must be allowed
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_histogram<kBlock, C, CHUNKED>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    });
    // about 8K keys per block (one batch per wave) for small n, at most four
    // blocks per CU for large n
    const uint32_t grid = grid_for(n, 8192, static_cast<uint32_t>(device_cu_count()) * 4);
    hipLaunchKernelGGL((k_histogram<kBlock, C, CHUNKED>), dim3(grid), dim3(kBlock), lds, stream, keys, n, ha,
                       hist);
}

template <bool CHUNKED>
static void launch_histogram_kernel(const uint32_t *keys, uint32_t n, const HistArgs &ha, uint32_t *hist,
                                    hipStream_t stream) {
    switch (hist_copies(ha.total_bins)) {
        case 16: launch_histogram_copies<16, CHUNKED>(keys, n, ha, hist, stream); break;
        case 8: launch_histogram_copies<8, CHUNKED>(keys, n, ha, hist, stream); break;
        case 4: launch_histogram_copies<4, CHUNKED>(keys, n, ha, hist, stream); break;
        case 2: launch_histogram_copies<2, CHUNKED>(keys, n, ha, hist, stream); break;
        default: launch_histogram_copies<1, CHUNKED>(keys, n, ha, hist, stream); break;
    }
}

template <int CC>
static void launch_histogram_auto_copies(const uint32_t *keys, uint32_t n, const HistArgs &hp, const HistArgs &hc,
                                         const uint32_t *mode, uint32_t *hist, hipStream_t stream) {
    constexpr int kBlock = 512, kCP = 16;
    const size_t lds = std::max(static_cast<size_t>(kCP) * (hp.total_bins + 1),
                                static_cast<size_t>(CC) * (hc.total_bins + 1)) * sizeof(uint32_t);
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_histogram_auto<kBlock, kCP, CC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    });
    const uint32_t grid = grid_for(n, 8192, static_cast<uint32_t>(device_cu_count()) * 4);
    hipLaunchKernelGGL((k_histogram_auto<kBlock, kCP, CC>), dim3(grid), dim3(kBlock), lds, stream, keys, n, hp, hc,
                       mode, hist);
}

// Whether the sample kernel chooses between XCD chunks and one chain (it
// runs only where the plain counts have all 16 lane-class copies, which the
// histogram kernel that reads its choice needs); otherwise r.chunked stands.
static bool sample_decides(const Resolved &r, uint32_t n) {
    return r.probe && hist_copies(hist_args(r, n, false).total_bins) == 16;
}

// hist_zeroed: the caller has cleared the counters already.  chunked: the
// per-chunk counts of a sort with r.chunked, in place of the plain ones;
// with mode set (r.probe) the probe kernel chooses between the two and
// writes its choice to *mode.  Returns whether it did (else the counts are
// per chunk exactly when chunked is set).
bool launch_histograms(const uint32_t *keys, uint32_t n, const Resolved &r, uint32_t *hist, hipStream_t stream,
                       bool hist_zeroed, bool chunked, uint32_t *mode) {
    const HistArgs ha = hist_args(r, n, chunked);
    if (!hist_zeroed) {
        hipLaunchKernelGGL(k_fill_zero, dim3(16), dim3(256), 0, stream, hist,
                           static_cast<size_t>(r.num_passes) * kMaxRadix);
        prof_mark(stream, RT_KIND_FILL);
    }
    const HistArgs hp = hist_args(r, n, false);
    const bool probe = chunked && mode != nullptr && sample_decides(r, n);
    if (probe) {
        hipLaunchKernelGGL(k_chunk_probe<1024>, dim3(1), dim3(1024), 0, stream, keys, n, ha, mode);
        prof_mark(stream, RT_KIND_PROBE);
        switch (hist_copies(ha.total_bins)) {
            case 16: launch_histogram_auto_copies<16>(keys, n, hp, ha, mode, hist, stream); break;
            case 8: launch_histogram_auto_copies<8>(keys, n, hp, ha, mode, hist, stream); break;
            case 4: launch_histogram_auto_copies<4>(keys, n, hp, ha, mode, hist, stream); break;
            case 2: launch_histogram_auto_copies<2>(keys, n, hp, ha, mode, hist, stream); break;
            default: launch_histogram_auto_copies<1>(keys, n, hp, ha, mode, hist, stream); break;
        }
    } else if (chunked) {
        launch_histogram_kernel<true>(keys, n, ha, hist, stream);
    } else {
        launch_histogram_kernel<false>(keys, n, ha, hist, stream);
    }
    prof_mark(stream, RT_KIND_HISTOGRAM);
    return probe;
}

// The whole sort (direct == false) or one explicit pass (direct == true,
// user_* read and direct_out_* written).
void launch_sort(uint32_t *keys, uint32_t *vals, uint32_t n, const Resolved &r, const Layout &L, char *ws,
                 bool direct, uint32_t *direct_out_k, uint32_t *direct_out_v, hipStream_t stream,
                 uint32_t pass_kind) {
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(ws + L.ctr);
    uint32_t *base = reinterpret_cast<uint32_t *>(ws + L.base);
    SortPlan *plan = reinterpret_cast<SortPlan *>(ws + L.plan);
    char *status = ws + L.status;

    prof_begin(stream);
    // the histogram counters and the lookback words of every pass ("not
    // published") start at zero: one fill over both (adjacent in the layout)
    const size_t fill_words = (L.status + L.status_bytes - L.hist) / 4;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(fill_words, 256 * 16, 4096)), dim3(256), 0, stream, hist,
                       fill_words);
    prof_mark(stream, RT_KIND_FILL);
    uint32_t *mode = ctr + kMaxPasses + 1 + kMaxPasses * kChunks;
    // fused: the upfront read counts only the first pass's digit; each pass
    // counts the next one's
    Resolved rh = r;
    if (r.fused) rh.num_passes = 1;
    const bool probed = launch_histograms(keys, n, rh, hist, stream, true, r.chunked, r.probe ? mode : nullptr);

    PlanArgs a{};
    a.num_passes = r.num_passes;
    for (uint32_t p = 0; p < r.num_passes; ++p) {
        a.shift[p] = r.shift[p];
        a.width[p] = r.width[p];
    }
    a.no_skip = (r.flags & RT_FLAG_NO_SKIP) ? 1u : 0u;
    a.n = n;
    a.tile = static_cast<uint32_t>(r.block * r.ipt);
    a.chunked = r.chunked ? 1u : 0u;
    if (r.chunked) pos_bounds(n, r, a.pos_bound);
    a.cbase = reinterpret_cast<uint32_t *>(ws + L.cbase);
    a.chunk_ctr = ctr + kMaxPasses + 1;
    a.mode = probed ? mode : nullptr;
    a.user_k = keys;
    a.user_v = r.with_values ? vals : nullptr;
    if (direct) {
        a.t1_k = direct_out_k;
        a.t1_v = r.with_values ? direct_out_v : nullptr;
    } else {
        a.t1_k = reinterpret_cast<uint32_t *>(ws + L.t1k);
        a.t1_v = r.with_values ? reinterpret_cast<uint32_t *>(ws + L.t1v) : nullptr;
        a.t2_k = L.t2k ? reinterpret_cast<uint32_t *>(ws + L.t2k) : nullptr;
        a.t2_v = (L.t2v && r.with_values) ? reinterpret_cast<uint32_t *>(ws + L.t2v) : nullptr;
    }
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(256), 0, stream, a, hist, base, plan, ctr, direct ? 1u : 0u);
    prof_mark(stream, RT_KIND_PLAN);

    for (uint32_t p = 0; p < r.num_passes; ++p) {
        const bool count_next = r.fused && p + 1 < r.num_passes;
        launch_pass(bits_class_of(r.width[p]), r.block, r.ipt, L, r.with_values, r.flags, stream, plan,
                    static_cast<int>(p), n, status + L.status_pass[p], ctr, pass_kind + p,
                    count_next ? hist : nullptr);
        if (count_next) {  // the next pass's digit starts from what this pass counted
            hipLaunchKernelGGL(k_plan_fused, dim3(1), dim3(256), 0, stream, hist, base, p + 1, r.width[p + 1], n);
            prof_mark(stream, RT_KIND_PLAN);
        }
    }

    if (!direct && (r.num_passes == 1 || !(r.flags & RT_FLAG_NO_SKIP))) {
        const uint32_t grid_c = grid_for(n, 256 * 8, static_cast<uint32_t>(device_cu_count()) * 8);
        hipLaunchKernelGGL(k_copy_back, dim3(grid_c), dim3(256), 0, stream, plan, a.t1_k, a.t1_v, keys,
                           a.user_v, n);
        prof_mark(stream, RT_KIND_COPY_BACK);
    }
}

}  // namespace rt

// ===========================================================================
// C ABI
// ===========================================================================

using namespace rt;

static rt_status check_ranges(const uint32_t *keys, const uint32_t *vals, size_t n, const char *what) {
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "%s: n = %zu, the limit is 2^32 - 1", what, n);
    if (n < 2) return RT_OK;
    if (keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "%s: keys is NULL with n = %zu", what, n);
    if ((reinterpret_cast<uintptr_t>(keys) & 3u) || (vals && (reinterpret_cast<uintptr_t>(vals) & 3u)))
        return set_error(RT_ERR_INVALID_ARG, "%s: arrays must be 4-byte aligned", what);
    if (vals != nullptr) {
        const uintptr_t k0 = reinterpret_cast<uintptr_t>(keys), v0 = reinterpret_cast<uintptr_t>(vals);
        const uintptr_t bytes = n * sizeof(uint32_t);
        if (k0 < v0 + bytes && v0 < k0 + bytes)
            return set_error(RT_ERR_INVALID_ARG, "%s: keys and values overlap", what);
    }
    return RT_OK;
}

extern "C" rt_status rt_sort_pairs_ex(uint32_t *keys, uint32_t *vals, size_t n, const rt_config *cfg,
                                void *workspace, size_t workspace_bytes, hipStream_t stream) {
    rt_status s = check_ranges(keys, vals, n, "rt_sort_pairs_ex");
    if (s != RT_OK || n < 2) return s;
    Resolved r;
    s = resolve_config(cfg, n, vals != nullptr, &r);
    if (s != RT_OK) return s;
    const Layout L = make_layout(n, r, false);
    void *ws = workspace;
    if (ws != nullptr) {
        if (workspace_bytes < L.total)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort_pairs_ex: workspace of %zu bytes, %zu needed",
                             workspace_bytes, L.total);
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort_pairs_ex: workspace must be 256-byte aligned");
    } else {
        s = cached_workspace(L.total, stream, &ws);
        if (s != RT_OK) return s;
    }
    launch_sort(keys, vals, static_cast<uint32_t>(n), r, L, static_cast<char *>(ws), false, nullptr, nullptr,
                stream);
    s = finish_call(stream, "rt_sort_pairs_ex");
    if (s == RT_OK && ((r.flags & RT_FLAG_VALIDATE) || debug_sync_enabled())) {
        // wait for the sort and read its error word (a lookback that gave up)
        uint32_t err = 0;
        s = read_device_word(static_cast<char *>(ws) + L.ctr + sizeof(uint32_t) * kMaxPasses, stream, &err,
                             "rt_sort_pairs_ex");
        if (s == RT_OK && err) return set_error(RT_ERR_HIP, "rt_sort_pairs_ex: device error word 0x%x", err);
    }
    return s;
}

// ---------------------------------------------------------------------------
// the sort without allocation: a static device scratch array as workspace
// ---------------------------------------------------------------------------

// Workspace of rt_sort_pairs_noalloc: one array per device, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a host-side stand-in); it uses the device address
// noalloc_scratch() looked up once per device.
constexpr size_t kNoAllocScratchBytes = static_cast<size_t>(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its scratch
}  // namespace

// The current device's scratch address, looked up with that device current
// on the first call on it.
static rt_status noalloc_scratch(void **out, const char *what) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "%s: hipGetDevice: %s", what, hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return RT_OK;
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
        return set_error(RT_ERR_HIP, "%s: hipGetSymbolAddress(scratch): %s", what, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return RT_OK;
}

extern "C" rt_status rt_sort_pairs_noalloc(uint32_t *keys, uint32_t *vals, size_t n, const rt_config *cfg,
                                           hipStream_t stream) {
    rt_status s = check_ranges(keys, vals, n, "rt_sort_pairs_noalloc");
    if (s != RT_OK || n < 2) return s;
    Resolved r;
    s = resolve_config(cfg, n, vals != nullptr, &r);
    if (s != RT_OK) return s;
    const Layout L = make_layout(n, r, false);
    if (L.total > kNoAllocScratchBytes)
        return set_error(RT_ERR_TOO_LARGE,
                         "rt_sort_pairs_noalloc: %zu items need %zu bytes of workspace; the static scratch holds %zu "
                         "(use rt_sort_pairs_ex)",
                         n, L.total, kNoAllocScratchBytes);
    void *ws = nullptr;
    s = noalloc_scratch(&ws, "rt_sort_pairs_noalloc");
    if (s != RT_OK) return s;
    // every region that must start at zero (histograms, lookback words,
    // tile counters, error word) is cleared by the sort's own kernels
    launch_sort(keys, vals, static_cast<uint32_t>(n), r, L, static_cast<char *>(ws), false, nullptr, nullptr,
                stream);
    s = finish_call(stream, "rt_sort_pairs_noalloc");
    if (s == RT_OK && ((r.flags & RT_FLAG_VALIDATE) || debug_sync_enabled())) {
        uint32_t err = 0;
        s = read_device_word(static_cast<char *>(ws) + L.ctr + sizeof(uint32_t) * kMaxPasses, stream, &err,
                             "rt_sort_pairs_noalloc");
        if (s == RT_OK && err) return set_error(RT_ERR_HIP, "rt_sort_pairs_noalloc: device error word 0x%x", err);
    }
    return s;
}

extern "C" rt_status rt_sort_keys(uint32_t *keys, size_t n, hipStream_t stream) {
    return rt_sort_pairs_ex(keys, nullptr, n, nullptr, nullptr, 0, stream);
}

extern "C" rt_status rt_sort_pairs(uint32_t *keys, uint32_t *vals, size_t n, hipStream_t stream) {
    if (vals == nullptr && n >= 2 && n < (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_INVALID_ARG, "rt_sort_pairs: vals is NULL (use rt_sort_keys)");
    return rt_sort_pairs_ex(keys, vals, n, nullptr, nullptr, 0, stream);
}

extern "C" size_t rt_workspace_bytes(size_t n, int with_values, const rt_config *cfg) {
    if (n < 2 || n >= (static_cast<size_t>(1) << 32)) return 0;
    Resolved r;
    if (resolve_config(cfg, n, with_values, &r) != RT_OK) return 0;
    return make_layout(n, r, false).total;
}

extern "C" rt_status rt_digit_histograms(const uint32_t *keys, size_t n, const rt_config *cfg,
                                         uint32_t *hist, hipStream_t stream) {
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "rt_digit_histograms: n = %zu", n);
    if (hist == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_digit_histograms: hist is NULL");
    if (keys == nullptr && n > 0) return set_error(RT_ERR_INVALID_ARG, "rt_digit_histograms: keys is NULL");
    Resolved r;
    rt_status s = resolve_config(cfg, n < 2 ? 2 : n, 0, &r);
    if (s != RT_OK) return s;
    prof_begin(stream);
    launch_histograms(keys, static_cast<uint32_t>(n), r, hist, stream, false, false, nullptr);
    return finish_call(stream, "rt_digit_histograms");
}

extern "C" rt_status rt_chunk_decision(const uint32_t *keys, size_t n, int with_values, const rt_config *cfg,
                                       uint32_t *mode, hipStream_t stream) {
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "rt_chunk_decision: n = %zu", n);
    if (mode == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_chunk_decision: mode is NULL");
    if (keys == nullptr && n > 0) return set_error(RT_ERR_INVALID_ARG, "rt_chunk_decision: keys is NULL");
    Resolved r;
    rt_status s = resolve_config(cfg, n < 2 ? 2 : n, with_values, &r);
    if (s != RT_OK) return s;
    prof_begin(stream);
    if (n >= 2 && sample_decides(r, static_cast<uint32_t>(n))) {
        hipLaunchKernelGGL(k_chunk_probe<1024>, dim3(1), dim3(1024), 0, stream, keys, static_cast<uint32_t>(n),
                           hist_args(r, n, true), mode);
        prof_mark(stream, RT_KIND_PROBE);
    } else {
        hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, stream, mode, (n >= 2 && r.chunked) ? 1u : 0u);
    }
    return finish_call(stream, "rt_chunk_decision");
}

extern "C" rt_status rt_counting_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout,
                                      uint32_t *vout, size_t n, uint32_t shift, uint32_t width,
                                      hipStream_t stream) {
    if ((vin == nullptr) != (vout == nullptr))
        return set_error(RT_ERR_INVALID_ARG, "rt_counting_pass: vin and vout must both be set or both NULL");
    if (width < 1 || width > static_cast<uint32_t>(kMaxBits) || shift + width > 32)
        return set_error(RT_ERR_INVALID_ARG, "rt_counting_pass: digit [%u, %u) invalid", shift, shift + width);
    rt_status s = check_ranges(kin, vin, n, "rt_counting_pass");
    if (s != RT_OK) return s;
    if (n == 0) return RT_OK;
    if (kout == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_counting_pass: kout is NULL");
    {
        const uintptr_t bytes = n * sizeof(uint32_t);
        const uintptr_t ins[2] = {reinterpret_cast<uintptr_t>(kin), reinterpret_cast<uintptr_t>(vin)};
        const uintptr_t outs[2] = {reinterpret_cast<uintptr_t>(kout), reinterpret_cast<uintptr_t>(vout)};
        for (int i = 0; i < 2; ++i)
            for (int o = 0; o < 2; ++o)
                if (ins[i] && outs[o] && ins[i] < outs[o] + bytes && outs[o] < ins[i] + bytes)
                    return set_error(RT_ERR_INVALID_ARG, "rt_counting_pass: inputs and outputs overlap");
        if (vout && reinterpret_cast<uintptr_t>(kout) < reinterpret_cast<uintptr_t>(vout) + bytes &&
            reinterpret_cast<uintptr_t>(vout) < reinterpret_cast<uintptr_t>(kout) + bytes)
            return set_error(RT_ERR_INVALID_ARG, "rt_counting_pass: the outputs overlap");
    }
    if (n == 1) {
        hipError_t e = hipMemcpyAsync(kout, kin, 4, hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess && vin) e = hipMemcpyAsync(vout, vin, 4, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "rt_counting_pass: %s", hipGetErrorString(e));
        return finish_call(stream, "rt_counting_pass");
    }
    rt_config c{};
    rt_config t;
    tuned_config(n, vin != nullptr, &t);
    c.num_passes = 1;
    c.digit_bits[0] = width;
    c.block_threads = t.block_threads;
    c.items_per_thread = t.items_per_thread;
    if (!shape_supported(bits_class_of(width), static_cast<int>(c.block_threads),
                         static_cast<int>(c.items_per_thread))) {
        c.block_threads = 512;
        c.items_per_thread = 16;
    }
    c.flags = RT_FLAG_NO_SKIP;
    // resolve with a placeholder full-width layout, then set the real digit
    Resolved r{};
    r.num_passes = 1;
    r.shift[0] = shift;
    r.width[0] = width;
    r.block = static_cast<int>(c.block_threads);
    r.ipt = static_cast<int>(c.items_per_thread);
    r.flags = c.flags;
    r.with_values = vin != nullptr;
    if (!shape_supported(bits_class_of(width), r.block, r.ipt))
        return set_error(RT_ERR_UNSUPPORTED, "rt_counting_pass: no kernel for this shape");
    const Layout L = make_layout(n, r, true);
    void *ws = nullptr;
    s = cached_workspace(L.total, stream, &ws);
    if (s != RT_OK) return s;
    launch_sort(const_cast<uint32_t *>(kin), const_cast<uint32_t *>(vin), static_cast<uint32_t>(n), r, L,
                static_cast<char *>(ws), true, kout, vout, stream);
    return finish_call(stream, "rt_counting_pass");
}

extern "C" rt_status rt_copy(const void *src, void *dst, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return RT_OK;
    if (src == nullptr || dst == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_copy: NULL pointer");
    if (bytes & 3u) return set_error(RT_ERR_INVALID_ARG, "rt_copy: bytes must be a multiple of 4");
    const int cus = device_cu_count();
    prof_begin(stream);
    const bool v16 = !((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst) | bytes) & 15u);
    if (v16) {
        const size_t words = bytes / 16;
        hipLaunchKernelGGL(k_copy16, dim3(static_cast<uint32_t>((words + 255) / 256)), dim3(256), 0, stream,
                           static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), words);
    } else {
        const size_t words = bytes / 4;
        hipLaunchKernelGGL(k_copy4, dim3(grid_for(words, 256 * 4, static_cast<uint32_t>(cus) * 16)), dim3(256), 0,
                           stream, static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst), words);
    }
    prof_mark(stream, RT_KIND_COPY);
    return finish_call(stream, "rt_copy");
}

extern "C" rt_status rt_bandwidth_probe(const void *src, void *dst, size_t bytes, uint32_t kind, uint32_t *sink,
                                        hipStream_t stream) {
    if (kind > RT_PROBE_WRITE) return set_error(RT_ERR_INVALID_ARG, "rt_bandwidth_probe: unknown kind %u", kind);
    if (bytes == 0) return RT_OK;
    const bool reads = kind != RT_PROBE_WRITE, writes = kind != RT_PROBE_READ;
    if ((reads && src == nullptr) || (writes && dst == nullptr) || (kind == RT_PROBE_READ && sink == nullptr))
        return set_error(RT_ERR_INVALID_ARG, "rt_bandwidth_probe: NULL pointer");
    if ((bytes | (reads ? reinterpret_cast<uintptr_t>(src) : 0u) | (writes ? reinterpret_cast<uintptr_t>(dst) : 0u)) &
        15u)
        return set_error(RT_ERR_INVALID_ARG, "rt_bandwidth_probe: pointers and bytes must be multiples of 16");
    const size_t words = bytes / 16;
    const uint32_t cus = static_cast<uint32_t>(device_cu_count());
    // the grid-stride probes: 16 blocks of 256 threads per CU
    const uint32_t grid = grid_for(words, 256 * kProbeWords, cus * 16);
    prof_begin(stream);
    switch (kind) {
        case RT_PROBE_COPY:
            hipLaunchKernelGGL(k_copy16, dim3(static_cast<uint32_t>((words + 255) / 256)), dim3(256), 0, stream,
                               static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), words);
            break;
        case RT_PROBE_COPY_NT:
            hipLaunchKernelGGL(k_copy16_nt, dim3(grid), dim3(256), 0, stream, static_cast<const uint4 *>(src),
                               static_cast<uint4 *>(dst), words);
            break;
        case RT_PROBE_READ:
            hipLaunchKernelGGL(k_read16, dim3(grid), dim3(256), 0, stream, static_cast<const uint4 *>(src), sink,
                               words);
            break;
        default:
            hipLaunchKernelGGL(k_write16, dim3(grid), dim3(256), 0, stream, static_cast<uint4 *>(dst), words);
            break;
    }
    prof_mark(stream, RT_KIND_COPY);
    return finish_call(stream, "rt_bandwidth_probe");
}

extern "C" rt_status rt_generate(uint32_t *keys, uint32_t *vals, size_t n, const rt_gen_params *params,
                                 uint32_t value_base, hipStream_t stream) {
    if (n >= (static_cast<size_t>(1) << 32)) return set_error(RT_ERR_TOO_LARGE, "rt_generate: n = %zu", n);
    if (params == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_generate: params is NULL");
    if (params->dist > RT_DIST_ZIPF16) return set_error(RT_ERR_INVALID_ARG, "rt_generate: unknown dist %u", params->dist);
    if (n == 0) return RT_OK;
    if (keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_generate: keys is NULL");
    GenArgs g{};
    g.dist = params->dist;
    g.value_base = value_base;
    g.state = params->state;
    memcpy(g.dictionary, params->dictionary, sizeof g.dictionary);
    memcpy(g.thresholds, params->thresholds, sizeof g.thresholds);
    const uint32_t grid = grid_for(n, 256 * 4, static_cast<uint32_t>(device_cu_count()) * 16);
    prof_begin(stream);
    hipLaunchKernelGGL(k_generate, dim3(grid), dim3(256), 0, stream, keys, vals, static_cast<uint32_t>(n), g);
    prof_mark(stream, RT_KIND_GENERATE);
    return finish_call(stream, "rt_generate");
}

extern "C" const char *rt_status_string(rt_status s) {
    switch (s) {
        case RT_OK: return "ok";
        case RT_ERR_INVALID_ARG: return "invalid argument";
        case RT_ERR_TOO_LARGE: return "too large";
        case RT_ERR_OUT_OF_MEMORY: return "out of memory";
        case RT_ERR_HIP: return "HIP error";
        case RT_ERR_BUDGET: return "over the HBM budget";
        case RT_ERR_UNSUPPORTED: return "unsupported";
        case RT_ERR_CANCELLED: return "cancelled";
        case RT_ERR_TIMEOUT: return "timed out";
        case RT_ERR_NOT_FOUND: return "not found";
    }
    return "unknown status";
}

extern "C" const char *rt_last_error(void) { return rt::last_error(); }

extern "C" const char *rt_version(void) { return "rtsort 0.1 (gfx950)"; }

extern "C" rt_status rt_profile_start(uint32_t max_marks) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (hipEvent_t e : g_prof_events) (void)hipEventDestroy(e);
    g_prof_events.clear();
    g_prof_marks.clear();
    g_prof_on.store(false);
    if (max_marks == 0) return RT_OK;
    g_prof_events.reserve(max_marks);
    g_prof_marks.reserve(max_marks);
    for (uint32_t i = 0; i < max_marks; ++i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) {
            for (hipEvent_t x : g_prof_events) (void)hipEventDestroy(x);
            g_prof_events.clear();
            return set_error(RT_ERR_HIP, "rt_profile_start: hipEventCreate: %s", hipGetErrorString(err));
        }
        g_prof_events.push_back(e);
    }
    g_prof_on.store(true);
    return RT_OK;
}

extern "C" rt_status rt_profile_stop(uint32_t *kinds, float *ms, uint32_t capacity, uint32_t *count) {
    g_prof_on.store(false);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    uint32_t out = 0;
    rt_status st = RT_OK;
    for (size_t i = 0; i < g_prof_marks.size(); ++i) {
        const Mark &m = g_prof_marks[i];
        // the previous mark on the same stream ends where this kernel starts
        // (for a call-start mark: the idle gap since the previous call)
        size_t j = i;
        while (j > 0 && g_prof_marks[j - 1].stream != m.stream) --j;
        hipError_t e = hipEventSynchronize(m.ev);
        float t = 0.f;
        if (e == hipSuccess && j > 0) e = hipEventElapsedTime(&t, g_prof_marks[j - 1].ev, m.ev);
        if (e != hipSuccess) {
            st = set_error(RT_ERR_HIP, "rt_profile_stop: %s", hipGetErrorString(e));
            break;
        }
        if (out < capacity) {
            if (kinds) kinds[out] = m.kind;
            if (ms) ms[out] = t;
        }
        ++out;
    }
    if (count) *count = out < capacity ? out : capacity;
    for (hipEvent_t e : g_prof_events) (void)hipEventDestroy(e);
    g_prof_events.clear();
    g_prof_marks.clear();
    return st;
}
