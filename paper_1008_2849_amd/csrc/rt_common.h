// rt_common.h -- host-side declarations shared by the library's sources.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "rt_internal.h"

// Tile shapes (digit bits class, threads per block, items per thread) for
// which onesweep kernels are compiled.  512 x 32 (16K items, two blocks per
// CU) is built for the staged pass with plain stores only.
#define RT_FOR_EACH_SHAPE(X) \
    X(8, 256, 16)            \
    X(8, 512, 16)            \
    X(8, 1024, 8)            \
    X(8, 1024, 12)           \
    X(8, 1024, 16)           \
    X(8, 512, 32)            \
    X(11, 256, 16)           \
    X(11, 512, 8)            \
    X(11, 512, 16)

namespace rt {

// A validated sort configuration.
struct Resolved {
    uint32_t num_passes;
    uint32_t shift[kMaxPasses];
    uint32_t width[kMaxPasses];
    int block;
    int ipt;
    uint32_t flags;
    bool with_values;
    bool chunked;  // passes may run in XCD chunks (every digit of at most 8 bits)
    bool probe;    // chunked: the probe kernel decides per sort (else chunks always)
    bool fused;    // RT_FLAG_FUSED_HISTOGRAM: passes count the next pass's digit
};

// Byte offsets of the workspace regions.
struct Layout {
    size_t hist, base, cbase, plan, ctr, status, status_bytes;
    size_t status_pass[kMaxPasses];
    size_t t1k, t1v, t2k, t2v;
    size_t total;
    uint32_t tiles;       // tiles of the global grid per pass
    uint32_t grid_tiles;  // blocks per pass: the grid cut at up to kChunks - 1 chunk ends
    bool wide_status;     // n >= 2^30: 64-bit lookback words and byte offsets
};

rt_status set_error(rt_status s, const char *fmt, ...);
const char *last_error();
bool debug_sync_enabled();
rt_status finish_call(hipStream_t stream, const char *what);
int device_cu_count();

bool shape_supported(int bits_class, int block, int ipt);

// Histogram arguments of a sort (32- or 64-bit keys) and the first pass's
// positional XCD chunks: chunk x reads input items [bound[x], bound[x + 1]),
// whole tiles, kChunks nearly equal shares of the tile grid.  chunked:
// per-chunk counts (see k_histogram).
struct HistArgs;
void pos_bounds(size_t n, const Resolved &r, uint32_t bound[kChunks + 1]);
HistArgs hist_args(const Resolved &r, size_t n, bool chunked);
rt_status resolve_config(const rt_config *cfg, size_t n, int with_values, Resolved *out);
Layout make_layout(size_t n, const Resolved &r, bool direct);
rt_status cached_workspace(size_t bytes, hipStream_t stream, void **out);
// Waits for the stream, then copies one u32 of device memory to *out.
rt_status read_device_word(const void *word, hipStream_t stream, uint32_t *out, const char *what);
// The whole sort (direct == false) or one explicit pass (direct == true:
// keys/vals read, direct_out_* written).  Pass p's timing mark has kind
// pass_kind + p.  After the plan kernel, the workspace's base table holds
// pass p's exclusive digit offsets at p * kMaxRadix, with every bin past the
// digit's range equal to n.
void launch_sort(uint32_t *keys, uint32_t *vals, uint32_t n, const Resolved &r, const Layout &L, char *ws,
                 bool direct, uint32_t *direct_out_k, uint32_t *direct_out_v, hipStream_t stream,
                 uint32_t pass_kind = RT_KIND_PASS);

// Whole-in-LDS kernel shapes (threads, items per thread, digit bits)
// compiled for the segmented sort; a shape holds segments of up to threads
// x items.  8-bit digits sort a 32-bit key in four passes, 11-bit digits in
// three (11, 11, 10); the 11-bit per-wave counters (8 KiB a wave) limit
// those to 512 threads.
#define RT_FOR_EACH_SEG_SMALL_SHAPE(X) \
    X(64, 4, 8)                        \
    X(64, 8, 8)                        \
    X(128, 4, 8)                       \
    X(128, 8, 8)                       \
    X(256, 4, 8)                       \
    X(256, 8, 8)                       \
    X(512, 4, 8)                       \
    X(512, 8, 8)                       \
    X(256, 16, 8)                      \
    X(128, 9, 8)                       \
    X(256, 9, 8)                       \
    X(256, 17, 8)                      \
    X(512, 16, 8)                      \
    X(1024, 8, 8)                      \
    X(1024, 16, 8)                     \
    X(64, 4, 11)                       \
    X(64, 8, 11)                       \
    X(128, 4, 11)                      \
    X(128, 8, 11)                      \
    X(256, 4, 11)                      \
    X(256, 8, 11)                      \
    X(256, 16, 11)                     \
    X(512, 4, 11)                      \
    X(512, 8, 11)                      \
    X(512, 16, 11)

// Tile shapes (threads, items per thread) of the tiled segments' passes.
#define RT_FOR_EACH_SEG_TILE_SHAPE(X) \
    X(1024, 16)                       \
    X(512, 16)

// The whole-in-LDS size classes of the segmented sort: class c holds the
// segments of more than cls[c - 1].max_n and at most cls[c].max_n items and
// sorts each with one block of the given shape.  Built in: up to 2048 items
// with 256x8, up to 8192 with 512x16, up to 16384 with 1024x16; a tuning
// table's "segments" entries replace it.
struct SegClass {
    uint32_t max_n;
    int block, ipt;
    int bits;  // digit width of the class's passes: 8 or 11
};
// The classes, and the tile shape (tile_block x tile_ipt items) of the
// tiled segments' passes (the server keeps 1024 x 16).
struct SegClassTable {
    uint32_t count;
    SegClass cls[kSegMaxClasses];
    int tile_block, tile_ipt;
    SegClassLimits limits() const;
    uint32_t lds_max() const { return count ? cls[count - 1].max_n : 0u; }
    uint32_t tile() const { return static_cast<uint32_t>(tile_block * tile_ipt); }
};
SegClassTable seg_class_table();
bool seg_small_shape_supported(int block, int ipt, int bits);
bool seg_tile_shape_supported(int block, int ipt);
// Launches the whole-in-LDS kernel of class `which` over its list; the
// segments are sorted on their low `key_bits` bits.
void launch_seg_small(const SegClass &c, bool vals, uint32_t max_listed, hipStream_t stream,
                      const SegDesc *descs, const uint32_t *list, const SegHeader *h, int which, int key_bits,
                      int to_temp);

// Workspace of a segmented sort (byte offsets) and its device pointers.
struct SegLayout {
    uint32_t num_segments;
    size_t capacity;          // temporaries hold this many items
    uint32_t large_capacity;  // most segments the tiled path can hold
    uint32_t max_tiles;
    uint32_t tile;            // items per tile of the tiled segments' passes
    bool wide_status;
    SegClassTable classes;    // size classes the layout was made for
    size_t header, descs, lists, first_tile, tile_seg, hist, base, status, status_pass, tk, tv;
    size_t total;
};

// Chunks of a segmented pass's tile list: kChunks when the segments hold
// kSegChunkMinTiles tiles or more on average (items / segments) and there
// are at least kSegChunkMinSegments of them, else 1.  Chunks end at segment
// ends, so they balance only with many segments per chunk; short segments
// (many partial tiles, short lookback chains) measured faster on one chain.
constexpr uint32_t kSegChunkMinTiles = 16;
constexpr uint32_t kSegChunkMinSegments = 16 * kChunks;
inline uint32_t seg_chunk_count(size_t items, size_t segments, uint32_t tile) {
    return segments >= kSegChunkMinSegments && items / segments >= static_cast<size_t>(kSegChunkMinTiles) * tile
               ? kChunks
               : 1u;
}

struct SegPointers {
    SegHeader *header;
    uint32_t *header_words;
    SegDesc *descs;
    uint32_t *lists;
    uint32_t *first_tile;
    SegDesc *tile_seg;  // per tile: its segment's descriptor, pad = the segment's first tile
    uint32_t *hist;
    uint32_t *base;
    char *status;
    uint32_t *tk;
    uint32_t *tv;
};

// own_temps: the workspace holds the temporaries (capacity items each);
// otherwise the caller supplies them.  The layout takes the current size
// classes (or `classes` when given), and a call uses those of its layout;
// tiled_only: none, every segment of two or more items goes through the
// tiled passes.
SegLayout make_seg_layout(uint32_t num_segments, size_t capacity, bool with_values, bool own_temps,
                          bool tiled_only = false, const SegClassTable *classes = nullptr);
SegPointers seg_pointers(char *ws, const SegLayout &L);
// Sorts segment s = [offsets[s], offsets[s+1]) of keys/vals on digits
// digit0..digit0 + passes - 1 with temporaries tk/tv at the same distance
// from offsets[0]; an even pass count leaves the result in keys/vals, an odd
// one (to_temp set) in tk/tv.  digit0 > 0 needs a tiled_only layout (the
// whole-in-LDS classes sort from digit 0).  persistent: the tiled passes run
// one block per CU that claims tiles until none is left, for calls whose
// tiled segments are usually few.
void launch_segments(uint32_t *keys, uint32_t *vals, uint32_t *tk, uint32_t *tv, const uint32_t *offsets,
                     uint32_t num_segments, const SegLayout &L, char *ws, int passes, int to_temp,
                     hipStream_t stream, uint32_t digit0 = 0, bool persistent = false);
void launch_batched(uint32_t *keys, uint32_t *vals, const uint32_t *offsets, uint32_t num_segments,
                    const SegLayout &L, char *ws, hipStream_t stream);

// Kernel timing marks (see rt_profile_start); cheap no-ops when disabled.
void prof_begin(hipStream_t stream);
void prof_mark(hipStream_t stream, uint32_t kind);

// Tuned configuration for n items (from the loaded table, else built in).
void tuned_config(size_t n, int with_values, rt_config *out);

}  // namespace rt
