// rt_sort64.hip -- host side of the LSD radix sort of 64-bit keys: argument
// checks, configuration, workspace layout, launch sequence and the C ABI.
// The planning kernel, the lookback words and the buffer scheme are those of
// the 32-bit sort; keys are 8 bytes and values 0, 4 or 8 bytes per item.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "rt_common.h"
#include "rt_wide_kernels.h"

// Tile shapes (digit bits class, threads, items per thread) compiled for
// 64-bit keys.  Tiles hold 8K items for 8-bit digits and 4K for 11-bit
// ones, so that keys, two value words and the per-wave counters fit in LDS.
// (4K-item tiles for 8-bit digits, 512x8 and 256x16, measured 10-25 %
// slower than both 8K shapes for every value width.)
#define RT64_FOR_EACH_SHAPE(X) \
    X(8, 1024, 8)              \
    X(8, 1024, 12)             \
    X(8, 1024, 16)             \
    X(8, 512, 16)              \
    X(11, 512, 8)

namespace rt {

namespace {

size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

bool shape64_supported(int bits_class, int block, int ipt) {
#define RT_SHAPE_CASE(B, BLK, I) \
    if (bits_class == B && block == BLK && ipt == I) return true;
    RT64_FOR_EACH_SHAPE(RT_SHAPE_CASE)
#undef RT_SHAPE_CASE
    return false;
}

int bits_class_of(uint32_t width) { return width <= 8 ? 8 : 11; }

// Built-in default: eight 8-bit digits.  From 2^24 items, 16K-item tiles
// (1024x16; with 8-byte values 1024x12), whose keys and values are staged
// one after the other when they do not fit the LDS together.  Measured at
// 2^28 items, pass times against the 8K-item shapes below: keys only 0.94
// vs 1.05-1.09 ms, 4-byte values 1.29-1.32 vs 1.55 ms, 8-byte values
// 1.67 vs 1.80-1.83 ms.  Below 2^24 items, 8K-item tiles (a grid of at
// least a few tiles per CU): 1024x8 for 4-byte values, else 512x16, whose
// LDS footprint without values (74 KiB) lets two blocks share a CU.
// 11-bit digits are 4-5x slower: a 4K-item tile publishes 2048 lookback
// words, more status traffic than data.
constexpr size_t kWideTileMinItems = static_cast<size_t>(1) << 24;

void default_config64(uint32_t value_words, size_t n, rt_config *c) {
    memset(c, 0, sizeof *c);
    c->num_passes = 8;
    for (int p = 0; p < 8; ++p) c->digit_bits[p] = 8;
    if (n >= kWideTileMinItems) {
        c->block_threads = 1024;
        c->items_per_thread = value_words == 2 ? 12 : 16;
    } else {
        c->block_threads = value_words == 1 ? 1024 : 512;
        c->items_per_thread = value_words == 1 ? 8 : 16;
    }
}

rt_status resolve64(const rt_config *cfg, uint32_t value_words, size_t n, Resolved *out) {
    rt_config c;
    default_config64(value_words, n, &c);
    if (cfg != nullptr && cfg->num_passes != 0) {
        c.num_passes = cfg->num_passes;
        memcpy(c.digit_bits, cfg->digit_bits, sizeof c.digit_bits);
    }
    if (cfg != nullptr) {
        c.flags = cfg->flags;
        if (cfg->block_threads) c.block_threads = cfg->block_threads;
        if (cfg->items_per_thread) c.items_per_thread = cfg->items_per_thread;
    }
    if (c.flags & ~static_cast<uint32_t>(RT_FLAG_NO_SKIP | RT_FLAG_ONE_CHAIN | RT_FLAG_CHUNKS | RT_FLAG_VALIDATE))
        return set_error(RT_ERR_UNSUPPORTED,
                         "64-bit keys: only RT_FLAG_NO_SKIP, RT_FLAG_ONE_CHAIN, RT_FLAG_CHUNKS and RT_FLAG_VALIDATE "
                         "are supported (flags 0x%x)",
                         c.flags);
    if ((c.flags & RT_FLAG_ONE_CHAIN) && (c.flags & RT_FLAG_CHUNKS))
        return set_error(RT_ERR_INVALID_ARG, "RT_FLAG_ONE_CHAIN and RT_FLAG_CHUNKS exclude each other");
    if (c.num_passes < 1 || c.num_passes > kMaxPasses)
        return set_error(RT_ERR_INVALID_ARG, "num_passes %u outside 1..%d", c.num_passes, kMaxPasses);
    Resolved r{};
    r.num_passes = c.num_passes;
    uint32_t total = 0;
    bool wide = false;
    for (uint32_t p = 0; p < c.num_passes; ++p) {
        const uint32_t w = c.digit_bits[p];
        if (w < 1 || w > static_cast<uint32_t>(kMaxBits))
            return set_error(RT_ERR_INVALID_ARG, "digit_bits[%u] = %u outside 1..%d", p, w, kMaxBits);
        r.shift[p] = total;
        r.width[p] = w;
        total += w;
        wide = wide || w > 8;
    }
    if (total != 64) return set_error(RT_ERR_INVALID_ARG, "digit widths sum to %u, not 64", total);
    r.block = static_cast<int>(c.block_threads);
    r.ipt = static_cast<int>(c.items_per_thread);
    const bool explicit_shape = cfg != nullptr && cfg->block_threads != 0 && cfg->items_per_thread != 0;
    if (!explicit_shape && wide) {  // the only shape built for wider digits
        r.block = 512;
        r.ipt = 8;
    }
    for (uint32_t p = 0; p < r.num_passes; ++p)
        if (!shape64_supported(bits_class_of(r.width[p]), r.block, r.ipt))
            return set_error(RT_ERR_UNSUPPORTED, "64-bit keys: no kernel for %d-bit digits with %d threads x %d items",
                             bits_class_of(r.width[p]), r.block, r.ipt);
    r.flags = c.flags;
    r.with_values = value_words > 0;
    *out = r;
    return RT_OK;
}

// XCD chunks for a sort of n items (as for 32-bit keys: digits of at most 8
// bits, the probe from kChunkMinItems items unless a flag decides).
void chunk_mode64(size_t n, Resolved *r) {
    const bool forced = (r->flags & RT_FLAG_CHUNKS) != 0;
    r->chunked = !(r->flags & RT_FLAG_ONE_CHAIN) && (forced || n >= kChunkMinItems);
    for (uint32_t p = 0; p < r->num_passes; ++p) r->chunked = r->chunked && r->width[p] <= 8;
    r->probe = r->chunked && !forced;
}

int copies64(uint32_t bins);

// Whether the sample kernel chooses between XCD chunks and one chain: only
// where the plain eight-digit counts have all 8 copies, as the histogram
// kernel that reads its choice needs; otherwise r.chunked stands.
static bool sample_decides64(const Resolved &r, uint32_t n) {
    return r.probe && copies64(hist_args(r, n, false).total_bins) == 8;
}

struct Layout64 {
    size_t hist, ctr, base, plan, status, status_bytes;
    size_t status_pass[kMaxPasses];
    size_t t1k, t1v, t2k, t2v;
    size_t cbase;
    size_t total;
    uint32_t tiles;
    uint32_t grid_tiles;  // blocks per pass: the grid cut at up to kChunks - 1 chunk ends
    bool wide_status;
};

Layout64 make_layout64(size_t n, const Resolved &r, uint32_t value_words) {
    Layout64 L{};
    const size_t tile = static_cast<size_t>(r.block) * r.ipt;
    const size_t tiles = (n + tile - 1) / tile;
    L.tiles = static_cast<uint32_t>(tiles);
    L.grid_tiles = static_cast<uint32_t>(tiles + (r.chunked ? kChunks - 1 : 0));
    L.wide_status = n >= (static_cast<size_t>(1) << 30);
    const size_t sw = L.wide_status ? 8 : 4;
    // the histograms (plain or per chunk) and the lookback words are
    // adjacent: one fill clears both
    size_t off = 0;
    L.hist = off;  off += align256(sizeof(uint32_t) * kMaxPasses * kMaxRadix);
    L.status = off;
    for (uint32_t p = 0; p < r.num_passes; ++p) {
        L.status_pass[p] = off - L.status;
        off += L.grid_tiles * (static_cast<size_t>(1) << (r.width[p] <= 8 ? 8 : 11)) * sw;
    }
    off = align256(off);
    L.status_bytes = off - L.status;
    // tile counters, the error word, kChunks tile counters per pass, the probe's choice
    L.ctr = off;   off += align256(sizeof(uint32_t) * (kMaxPasses + 2 + kMaxPasses * kChunks));
    L.base = off;  off += align256(sizeof(uint32_t) * kMaxPasses * kMaxRadix);
    L.cbase = off; off += align256(sizeof(uint32_t) * kMaxPasses * kChunks * kChunkRadix);
    L.plan = off;  off += align256(sizeof(SortPlan));
    const bool need_t2 = (r.num_passes & 1u) || !(r.flags & RT_FLAG_NO_SKIP);
    const size_t karr = align256(n * sizeof(uint64_t));
    const size_t varr = align256(n * sizeof(uint32_t) * value_words);
    L.t1k = off; off += karr;
    L.t1v = 0;
    if (value_words) { L.t1v = off; off += varr; }
    L.t2k = L.t2v = 0;
    if (need_t2) {
        L.t2k = off; off += karr;
        if (value_words) { L.t2v = off; off += varr; }
    }
    L.total = off;
    return L;
}

uint32_t grid_for(size_t items, size_t per_block, uint32_t cap) {
    size_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<uint32_t>(g);
}

// lane-class copies: as many as fit in 72 KiB of padded rows, at most 8
int copies64(uint32_t bins) {
    int c = 8;
    while (c > 1 && static_cast<size_t>(c) * (bins + 1) * sizeof(uint32_t) > 72 * 1024) c /= 2;
    return c;
}

template <int C>
void launch_histogram64_chunked(const uint64_t *keys, uint32_t n, const HistArgs &hc, uint32_t *hist,
                                hipStream_t stream) {
    constexpr int kBlock = 512;
    const size_t lds = static_cast<size_t>(C) * (hc.total_bins + 1) * sizeof(uint32_t);
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_histogram64_chunked<kBlock, C>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    });
    const uint32_t grid = grid_for(n, 4096, static_cast<uint32_t>(device_cu_count()) * 4);
    hipLaunchKernelGGL((k_histogram64_chunked<kBlock, C>), dim3(grid), dim3(kBlock), lds, stream, keys, n, hc, hist);
}

template <int CC>
void launch_histogram64_auto(const uint64_t *keys, uint32_t n, const HistArgs &hp, const HistArgs &hc,
                             const uint32_t *mode, uint32_t *hist, hipStream_t stream) {
    constexpr int kBlock = 512, kCP = 8;
    const size_t lds = std::max(static_cast<size_t>(kCP) * (hp.total_bins + 1),
                                static_cast<size_t>(CC) * (hc.total_bins + 1)) * sizeof(uint32_t);
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_histogram64_auto<kBlock, kCP, CC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    });
    const uint32_t grid = grid_for(n, 4096, static_cast<uint32_t>(device_cu_count()) * 4);
    hipLaunchKernelGGL((k_histogram64_auto<kBlock, kCP, CC>), dim3(grid), dim3(kBlock), lds, stream, keys, n, hp, hc,
                       mode, hist);
}

template <int C>
void launch_histogram64_copies(const uint64_t *keys, uint32_t n, const HistArgs &ha, uint32_t *hist,
                               hipStream_t stream) {
    constexpr int kBlock = 512;
    const size_t lds = static_cast<size_t>(C) * (ha.total_bins + 1) * sizeof(uint32_t);
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_histogram64<kBlock, C>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
    });
    const uint32_t grid = grid_for(n, 4096, static_cast<uint32_t>(device_cu_count()) * 4);
    hipLaunchKernelGGL((k_histogram64<kBlock, C>), dim3(grid), dim3(kBlock), lds, stream, keys, n, ha, hist);
}

template <int BITS, int BLOCK, int IPT>
void launch_pass64_shape(const Layout64 &L, uint32_t vw, hipStream_t stream, const SortPlan *plan, int pass,
                         uint32_t n, void *status, uint32_t *ctr) {
    const dim3 grid(L.grid_tiles), block(BLOCK);
    uint32_t *err = ctr + kMaxPasses;
    uint32_t *chunk_ctr = ctr + kMaxPasses + 1 + pass * kChunks;
#define RT_OS64(V, S)                                                                                      \
    hipLaunchKernelGGL((k_onesweep64<BITS, BLOCK, IPT, V, S>), grid, block, 0, stream, plan, pass, n, \
                       static_cast<S *>(status), chunk_ctr, err)
    if (L.wide_status) {
        if (vw == 2) RT_OS64(2, uint64_t); else if (vw == 1) RT_OS64(1, uint64_t); else RT_OS64(0, uint64_t);
    } else {
        if (vw == 2) RT_OS64(2, uint32_t); else if (vw == 1) RT_OS64(1, uint32_t); else RT_OS64(0, uint32_t);
    }
#undef RT_OS64
    prof_mark(stream, RT_KIND_PASS + pass);
}

void launch_pass64(int bits_class, int block, int ipt, const Layout64 &L, uint32_t vw, hipStream_t stream,
                   const SortPlan *plan, int pass, uint32_t n, void *status, uint32_t *ctr) {
#define RT_SHAPE_LAUNCH(B, BLK, I)                                                    \
    if (bits_class == B && block == BLK && ipt == I) {                                \
        launch_pass64_shape<B, BLK, I>(L, vw, stream, plan, pass, n, status, ctr);    \
        return;                                                                       \
    }
    RT64_FOR_EACH_SHAPE(RT_SHAPE_LAUNCH)
#undef RT_SHAPE_LAUNCH
}

void launch_sort64(uint64_t *keys, uint32_t *vals, uint32_t vw, uint32_t n, const Resolved &r, const Layout64 &L,
                   char *ws, hipStream_t stream) {
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    uint32_t *ctr = reinterpret_cast<uint32_t *>(ws + L.ctr);
    uint32_t *base = reinterpret_cast<uint32_t *>(ws + L.base);
    SortPlan *plan = reinterpret_cast<SortPlan *>(ws + L.plan);
    char *status = ws + L.status;
    const uint32_t cus = static_cast<uint32_t>(device_cu_count());

    prof_begin(stream);
    // histogram counters and lookback words, adjacent in the layout
    const size_t fill_words = (L.status + L.status_bytes - L.hist) / 4;
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(fill_words, 256 * 16, 4096)), dim3(256), 0, stream, hist,
                       fill_words);
    prof_mark(stream, RT_KIND_FILL);

    const HistArgs ha = hist_args(r, n, false);
    uint32_t *mode = ctr + kMaxPasses + 1 + kMaxPasses * kChunks;
    uint32_t pos_bound[kChunks + 1] = {};
    if (r.chunked) pos_bounds(n, r, pos_bound);
    bool probed = false;
    if (r.chunked) {
        const HistArgs hc = hist_args(r, n, true);
        if (sample_decides64(r, n)) {
            hipLaunchKernelGGL((k_chunk_probe<1024, uint64_t>), dim3(1), dim3(1024), 0, stream, keys, n, hc, mode);
            prof_mark(stream, RT_KIND_PROBE);
            switch (copies64(hc.total_bins)) {
                case 8: launch_histogram64_auto<8>(keys, n, ha, hc, mode, hist, stream); break;
                case 4: launch_histogram64_auto<4>(keys, n, ha, hc, mode, hist, stream); break;
                case 2: launch_histogram64_auto<2>(keys, n, ha, hc, mode, hist, stream); break;
                default: launch_histogram64_auto<1>(keys, n, ha, hc, mode, hist, stream); break;
            }
            probed = true;
        } else {
            switch (copies64(hc.total_bins)) {
                case 8: launch_histogram64_chunked<8>(keys, n, hc, hist, stream); break;
                case 4: launch_histogram64_chunked<4>(keys, n, hc, hist, stream); break;
                case 2: launch_histogram64_chunked<2>(keys, n, hc, hist, stream); break;
                default: launch_histogram64_chunked<1>(keys, n, hc, hist, stream); break;
            }
        }
    } else {
        switch (copies64(ha.total_bins)) {
            case 8: launch_histogram64_copies<8>(keys, n, ha, hist, stream); break;
            case 4: launch_histogram64_copies<4>(keys, n, ha, hist, stream); break;
            case 2: launch_histogram64_copies<2>(keys, n, ha, hist, stream); break;
            default: launch_histogram64_copies<1>(keys, n, ha, hist, stream); break;
        }
    }
    prof_mark(stream, RT_KIND_HISTOGRAM);

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
    for (int x = 0; x <= kChunks; ++x) a.pos_bound[x] = pos_bound[x];
    a.cbase = reinterpret_cast<uint32_t *>(ws + L.cbase);
    a.chunk_ctr = ctr + kMaxPasses + 1;
    a.mode = probed ? mode : nullptr;
    a.user_k = reinterpret_cast<uint32_t *>(keys);
    a.user_v = vw ? vals : nullptr;
    a.t1_k = reinterpret_cast<uint32_t *>(ws + L.t1k);
    a.t1_v = vw ? reinterpret_cast<uint32_t *>(ws + L.t1v) : nullptr;
    a.t2_k = L.t2k ? reinterpret_cast<uint32_t *>(ws + L.t2k) : nullptr;
    a.t2_v = (L.t2v && vw) ? reinterpret_cast<uint32_t *>(ws + L.t2v) : nullptr;
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(256), 0, stream, a, hist, base, plan, ctr, 0u);
    prof_mark(stream, RT_KIND_PLAN);

    for (uint32_t p = 0; p < r.num_passes; ++p)
        launch_pass64(bits_class_of(r.width[p]), r.block, r.ipt, L, vw, stream, plan, static_cast<int>(p), n,
                      status + L.status_pass[p], ctr);

    if (r.num_passes == 1 || !(r.flags & RT_FLAG_NO_SKIP)) {
        const uint32_t grid_c = grid_for(2 * static_cast<size_t>(n), 256 * 8, cus * 8);
        hipLaunchKernelGGL(k_copy_back_words, dim3(grid_c), dim3(256), 0, stream, plan, a.t1_k, a.t1_v,
                           a.user_k, a.user_v, 2 * static_cast<size_t>(n), static_cast<size_t>(vw) * n);
        prof_mark(stream, RT_KIND_COPY_BACK);
    }
}

rt_status check64(const uint64_t *keys, const void *vals, uint32_t value_bytes, size_t n, const char *what) {
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "%s: n = %zu, the limit is 2^32 - 1", what, n);
    if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8)
        return set_error(RT_ERR_INVALID_ARG, "%s: value_bytes = %u (0, 4 or 8)", what, value_bytes);
    if (n < 2) return RT_OK;
    if (keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "%s: keys is NULL with n = %zu", what, n);
    if (value_bytes != 0 && vals == nullptr)
        return set_error(RT_ERR_INVALID_ARG, "%s: vals is NULL with value_bytes = %u", what, value_bytes);
    if (reinterpret_cast<uintptr_t>(keys) & 7u)
        return set_error(RT_ERR_INVALID_ARG, "%s: keys must be 8-byte aligned", what);
    if (value_bytes != 0 && (reinterpret_cast<uintptr_t>(vals) & (value_bytes - 1)))
        return set_error(RT_ERR_INVALID_ARG, "%s: vals must be %u-byte aligned", what, value_bytes);
    if (value_bytes != 0) {
        const uintptr_t k0 = reinterpret_cast<uintptr_t>(keys), v0 = reinterpret_cast<uintptr_t>(vals);
        if (k0 < v0 + n * value_bytes && v0 < k0 + n * sizeof(uint64_t))
            return set_error(RT_ERR_INVALID_ARG, "%s: keys and values overlap", what);
    }
    return RT_OK;
}

}  // namespace

}  // namespace rt

using namespace rt;

extern "C" size_t rt_workspace_bytes64(size_t n, uint32_t value_bytes, const rt_config *cfg) {
    if (n < 2 || n >= (static_cast<size_t>(1) << 32)) return 0;
    if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8) return 0;
    Resolved r;
    if (resolve64(cfg, value_bytes / 4, n, &r) != RT_OK) return 0;
    chunk_mode64(n, &r);
    return make_layout64(n, r, value_bytes / 4).total;
}

extern "C" rt_status rt_sort64_ex(uint64_t *keys, void *vals, uint32_t value_bytes, size_t n, const rt_config *cfg,
                                  void *workspace, size_t workspace_bytes, hipStream_t stream) {
    rt_status s = check64(keys, vals, value_bytes, n, "rt_sort64_ex");
    if (s != RT_OK || n < 2) return s;
    const uint32_t vw = value_bytes / 4;
    Resolved r;
    s = resolve64(cfg, vw, n, &r);
    if (s == RT_OK) chunk_mode64(n, &r);
    if (s != RT_OK) return s;
    const Layout64 L = make_layout64(n, r, vw);
    void *ws = workspace;
    if (ws != nullptr) {
        if (workspace_bytes < L.total)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort64_ex: workspace of %zu bytes, %zu needed", workspace_bytes,
                             L.total);
        if (reinterpret_cast<uintptr_t>(ws) & 255u)
            return set_error(RT_ERR_INVALID_ARG, "rt_sort64_ex: workspace must be 256-byte aligned");
    } else {
        s = cached_workspace(L.total, stream, &ws);
        if (s != RT_OK) return s;
    }
    launch_sort64(keys, static_cast<uint32_t *>(vals), vw, static_cast<uint32_t>(n), r, L, static_cast<char *>(ws),
                  stream);
    s = finish_call(stream, "rt_sort64_ex");
    if (s == RT_OK && ((r.flags & RT_FLAG_VALIDATE) || debug_sync_enabled())) {
        uint32_t err = 0;
        s = read_device_word(static_cast<char *>(ws) + L.ctr + sizeof(uint32_t) * kMaxPasses, stream, &err,
                             "rt_sort64_ex");
        if (s == RT_OK && err) return set_error(RT_ERR_HIP, "rt_sort64_ex: device error word 0x%x", err);
    }
    return s;
}

extern "C" rt_status rt_chunk_decision64(const uint64_t *keys, size_t n, uint32_t value_bytes, const rt_config *cfg,
                                         uint32_t *mode, hipStream_t stream) {
    if (n >= (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_TOO_LARGE, "rt_chunk_decision64: n = %zu", n);
    if (mode == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_chunk_decision64: mode is NULL");
    if (keys == nullptr && n > 0) return set_error(RT_ERR_INVALID_ARG, "rt_chunk_decision64: keys is NULL");
    if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8)
        return set_error(RT_ERR_INVALID_ARG, "rt_chunk_decision64: value_bytes %u is not 0, 4 or 8", value_bytes);
    Resolved r;
    rt_status s = resolve64(cfg, value_bytes / 4, n, &r);
    if (s != RT_OK) return s;
    chunk_mode64(n, &r);
    prof_begin(stream);
    if (n >= 2 && sample_decides64(r, static_cast<uint32_t>(n))) {
        hipLaunchKernelGGL((k_chunk_probe<1024, uint64_t>), dim3(1), dim3(1024), 0, stream, keys,
                           static_cast<uint32_t>(n), hist_args(r, n, true), mode);
        prof_mark(stream, RT_KIND_PROBE);
    } else {
        hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, stream, mode, (n >= 2 && r.chunked) ? 1u : 0u);
    }
    return finish_call(stream, "rt_chunk_decision64");
}

extern "C" rt_status rt_sort_keys64(uint64_t *keys, size_t n, hipStream_t stream) {
    return rt_sort64_ex(keys, nullptr, 0, n, nullptr, nullptr, 0, stream);
}

extern "C" rt_status rt_sort_pairs64(uint64_t *keys, uint32_t *vals, size_t n, hipStream_t stream) {
    if (vals == nullptr && n >= 2 && n < (static_cast<size_t>(1) << 32))
        return set_error(RT_ERR_INVALID_ARG, "rt_sort_pairs64: vals is NULL (use rt_sort_keys64)");
    return rt_sort64_ex(keys, vals, 4, n, nullptr, nullptr, 0, stream);
}
