// rt_seg_kernels.h -- gfx950 kernels of the segmented (batched) sort.
//
// Many independent arrays ("segments": the slices of one batched call, or
// the requests of the server) are sorted together.  Each segment is
// described by a SegDesc; a work list picks the segments of a launch.
//
// * Segments of at most 16K items are sorted whole inside one block: one
//   read and one write of HBM, the four 8-bit counting-sort passes running
//   between LDS and registers.
// * Larger segments are cut into 16K-item tiles and sorted by per-segment
//   counting-sort passes in the onesweep form of rt_kernels.h: upfront
//   per-segment histograms, per-segment exclusive prefix sums, then per pass
//   one launch covering the tiles of every segment, with each segment's
//   lookback chain ending at its own first tile.
//
// Each pass is Section 3's counting sort (histogram, exclusive prefix sum,
// stable scatter) and the pass sequence is Section 4's LSD order; a segment
// is sorted exactly as a single array of its own would be.
#include "rt_kernels.h"

namespace rt {

// ---------------------------------------------------------------------------
// set-up of a batched call: descriptors and work lists from the offsets
// ---------------------------------------------------------------------------

static __global__ __launch_bounds__(64) void k_seg_reset(SegHeader *__restrict__ h) {
    uint32_t *w = reinterpret_cast<uint32_t *>(h);
    for (uint32_t i = threadIdx.x; i < sizeof(SegHeader) / 4; i += 64) w[i] = 0u;
}

// One thread per segment.  Segment s is [off[s], off[s+1]) of keys/vals; its
// temporaries sit at the same distance from off[0] in tk/tv, which hold
// `capacity` elements.  A segment with an end before its start, or reaching
// past off[0] + capacity, is left untouched and raises kSegErrBounds.  When
// the result is wanted in the temporaries (to_temp), a one-item segment is
// copied there here, as no later kernel sees it.  List slots are taken per
// wave: one atomic per class and wave, each lane's slot found from the
// class's ballot.
static __global__ __launch_bounds__(256) void k_seg_classify(const uint32_t *__restrict__ off, uint32_t num_segments,
                                                      uint32_t *keys, uint32_t *vals, uint32_t *tk, uint32_t *tv,
                                                      size_t capacity, uint32_t large_capacity, int to_temp,
                                                      SegClassLimits classes, SegDesc *__restrict__ descs,
                                                      uint32_t *__restrict__ lists, SegHeader *__restrict__ h) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    int c = -1;  // list of this lane's segment (-1: none)
    SegDesc d;
    if (s < num_segments) {
        const uint32_t o0 = off[0];
        const uint32_t a = off[s], b = off[s + 1];
        if (b < a || a < o0 || static_cast<size_t>(b - o0) > capacity) {
            atomicOr(&h->error, kSegErrBounds);
        } else if (b - a < 2) {  // nothing to sort
            if (b - a == 1 && to_temp) {
                tk[a - o0] = keys[a];
                if (vals) tv[a - o0] = vals[a];
            }
        } else {
            const uint32_t n = b - a;
            d.k = keys + a;
            d.v = vals ? vals + a : nullptr;
            d.tk = tk + (a - o0);
            d.tv = tv ? tv + (a - o0) : nullptr;
            d.n = n;
            d.pass = 0;
            d.row = 0;
            d.pad = 0;
            c = kSegLarge;
#pragma unroll
            for (int i = kSegMaxClasses - 1; i >= 0; --i)
                if (i < static_cast<int>(classes.count) && n <= classes.max_n[i]) c = i;
        }
    }
    uint32_t at = 0;
#pragma unroll
    for (int q = 0; q <= kSegLarge; ++q) {
        const uint64_t mine = __builtin_amdgcn_ballot_w64(c == q);
        if (mine == 0) continue;
        const uint32_t lane_lo = static_cast<uint32_t>(mine), lane_hi = static_cast<uint32_t>(mine >> 32);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(lane_hi, __builtin_amdgcn_mbcnt_lo(lane_lo, 0u));
        uint32_t first = 0;
        if (below == 0 && c == q) first = atomicAdd(&h->count[q], static_cast<uint32_t>(__popcll(mine)));
        // the wave's first lane of class q took the block of slots: share it
        const int leader = __builtin_ffsll(static_cast<long long>(mine)) - 1;
        first = __shfl(first, leader, 64);
        if (c == q) at = first + below;
    }
    if (c < 0) return;
    if (c == kSegLarge) {
        if (at >= large_capacity) {  // only if capacity does not bound the offsets
            atomicOr(&h->error, kSegErrBounds);
            return;
        }
        d.row = at;
    }
    descs[s] = d;
    lists[static_cast<size_t>(c) * num_segments + at] = s;
}

// The tiled list as the server builds it on the host has no counter on the
// device yet: this sets it.
static __global__ __launch_bounds__(64) void k_seg_set_count(SegHeader *__restrict__ h, int which, uint32_t count) {
    if (threadIdx.x == 0) h->count[which] = count;
}

// One block: first_tile[i] = tiles of list entries before i, and the total.
// Well-formed offsets never list more than large_capacity segments nor more
// than max_tiles tiles; overlapping (malformed) ones can, and then the list
// is cut to what the workspace holds (or emptied) and the error is raised,
// so that no later kernel indexes past the tables.
static __global__ __launch_bounds__(1024) void k_seg_tiles(const SegDesc *__restrict__ descs,
                                                           const uint32_t *__restrict__ list,
                                                           uint32_t *__restrict__ first_tile, SegHeader *__restrict__ h,
                                                           uint32_t large_capacity, uint32_t max_tiles, uint32_t tile) {
    __shared__ uint32_t s_wsum[16];
    const uint32_t listed = h->count[kSegLarge];
    const uint32_t count = min(listed, large_capacity);
    const uint32_t per = (count + 1023u) / 1024u;
    const uint32_t lo = min(count, threadIdx.x * per), hi = min(count, lo + per);
    uint32_t sum = 0;  // at most 256 entries of at most 2^19 tiles: no overflow
    for (uint32_t i = lo; i < hi; ++i) sum += (descs[list[i]].n + tile - 1) / tile;
    // saturate, so the block total stays exact up to max_tiles and cannot wrap
    uint32_t run = block_exclusive_sum<1024>(min(sum, max_tiles + 1u), s_wsum);
    for (uint32_t i = lo; i < hi; ++i) {
        first_tile[i] = run;
        run += (descs[list[i]].n + tile - 1) / tile;
    }
    if (threadIdx.x == 1023) {
        const bool fits = run <= max_tiles;
        first_tile[count] = run;
        h->count[kSegLarge] = fits ? count : 0u;
        h->total_tiles = fits ? run : 0u;
        if (!fits || listed != count) atomicOr(&h->error, kSegErrBounds);
    }
}

// Zeroes what a segmented call's counting and passes will use: the
// histogram rows of its listed tiled segments and, for each of `passes`
// passes, the lookback words of its tiles (both counts from k_seg_tiles),
// rather than the tables' full size, which holds the most tiled segments and
// tiles the workspace allows.  status_pass_words: one pass's region, in
// 32-bit words; word_u32s: 32-bit words per lookback word (1 or 2).
static __global__ __launch_bounds__(256) void k_seg_clear(const SegHeader *__restrict__ h,
                                                   uint32_t *__restrict__ hist, uint32_t *__restrict__ status,
                                                   size_t status_pass_words, uint32_t word_u32s, int passes) {
    const size_t hist_words = static_cast<size_t>(h->count[kSegLarge]) * kSegPasses * kSegRadix;
    const size_t status_words = static_cast<size_t>(h->total_tiles) * kSegRadix * word_u32s;
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    const size_t first = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    for (size_t i = first; i < hist_words; i += stride) hist[i] = 0u;
    for (int p = 0; p < passes; ++p)
        for (size_t i = first; i < status_words; i += stride) status[p * status_pass_words + i] = 0u;
}

// tile_desc[t] = the descriptor of the segment that tile t belongs to, with
// pad = that segment's first tile (first_tile is strictly increasing: every
// listed segment has at least one tile), so that a tile's kernel reaches its
// segment in one load rather than a chain of three.  Block 0 also cuts the
// tile list into nchunks (1 or kChunks) chunks of about equal tile counts at
// segment ends (a segment's tiles stay on one XCD).
static __global__ __launch_bounds__(256) void k_seg_tilemap(const SegDesc *__restrict__ descs,
                                                     const uint32_t *__restrict__ list,
                                                     const uint32_t *__restrict__ first_tile,
                                                     SegHeader *__restrict__ h,
                                                     SegDesc *__restrict__ tile_desc, uint32_t nchunks) {
    const uint32_t count = h->count[kSegLarge];
    const uint32_t total = h->total_tiles;
    if (blockIdx.x == 0 && threadIdx.x <= kChunks) {
        const uint32_t x = threadIdx.x;
        uint32_t at = total;
        if (x == 0) {
            at = 0;
        } else if (x < nchunks && count > 0) {
            // the first segment start at or after x / kChunks of the tiles
            const uint32_t target = static_cast<uint32_t>(static_cast<uint64_t>(x) * total / nchunks);
            uint32_t lo = 0, hi = count;  // first_tile[count] = total
            while (lo < hi) {
                const uint32_t mid = (lo + hi) / 2;
                if (first_tile[mid] >= target) hi = mid;
                else lo = mid + 1;
            }
            at = first_tile[lo];
        }
        h->chunk_start[x] = at;
    }
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < total; t += gridDim.x * 256) {
        uint32_t lo = 0, hi = count - 1;  // the last entry with first_tile <= t
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) / 2;
            if (first_tile[mid] <= t) lo = mid;
            else hi = mid - 1;
        }
        SegDesc d = descs[list[lo]];
        d.pad = first_tile[lo];
        tile_desc[t] = d;
    }
}

// ---------------------------------------------------------------------------
// whole segment in one block
// ---------------------------------------------------------------------------

// Sorts segments of at most BLOCK * IPT items, one per block at a time.  The
// segment is loaded once from k/v, taken through the digits of passes
// 0..passes-1 in LDS, and stored once: to k/v, or to tk/tv when to_temp is
// set (where the tiled passes leave an odd pass count's result).  Slots
// wholly past the segment's end are neither ranked nor staged; the empty
// lanes of the slot that holds the end take all-ones keys, which rank behind
// every real item (they come last in input order and the sort is stable),
// so the items' positions are those of the segment alone.  Ranking inside a
// pass is the onesweep ranking: wave-local ballot match plus per-wave digit
// counters, then digit offsets across the block.
template <int BLOCK, int IPT, bool VALS, int BITS>
__global__ __launch_bounds__(BLOCK) void k_seg_small(const SegDesc *__restrict__ descs,
                                                     const uint32_t *__restrict__ list,
                                                     const SegHeader *__restrict__ h, int which, int key_bits,
                                                     int to_temp) {
    constexpr int RADIX = 1 << BITS;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * IPT;
    constexpr int WAVE_ITEMS = 64 * IPT;
    constexpr int R = RADIX >= BLOCK ? RADIX / BLOCK : 1;
    constexpr int DT = RADIX / R;
    __shared__ uint32_t s_k[TILE];
    __shared__ uint32_t s_v[VALS ? TILE : 1];
    __shared__ uint32_t s_whist[WAVES * RADIX + WAVES * 64];
    __shared__ uint32_t s_wsum[WAVES];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t wslot0 = wave * WAVE_ITEMS + lane;
    uint32_t *wh = s_whist + wave * RADIX;
    uint32_t *scratch = s_whist + WAVES * RADIX + wave * 64 + lane;
    const uint32_t count = h->count[which];

    for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
        const SegDesc d = descs[list[e]];
        const uint32_t n = d.n;
        uint32_t key[IPT];
        uint32_t val[VALS ? IPT : 1];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = wslot0 + j * 64;
            key[j] = i < n ? d.k[i] : ~0u;
            if constexpr (VALS) val[j] = i < n ? d.v[i] : 0u;
        }
        for (uint32_t shift = 0; shift < static_cast<uint32_t>(key_bits); shift += BITS) {
            const uint32_t width = min(static_cast<uint32_t>(BITS), static_cast<uint32_t>(key_bits) - shift);
            for (uint32_t i = lane; i < RADIX; i += 64) wh[i] = 0u;
            // (the previous pass finished reading wh before its last barrier)
            uint32_t rnk[IPT];
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                if (wave * WAVE_ITEMS + j * 64 >= n) continue;  // a slot past the segment: no item to rank
                const uint32_t dg = __builtin_amdgcn_ubfe(key[j], shift, width);
                uint32_t lo, hi;
                match_digit<BITS>(dg, lo, hi);
                const uint32_t cnt = wh[dg];
                // mbcnt and bcnt add the counter while they count
                const uint32_t r = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, cnt));
                rnk[j] = r;
                uint32_t *dst = r == cnt ? wh + dg : scratch;
                uint32_t t;
                asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(t) : "v"(lo), "v"(cnt));
                asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(t) : "v"(hi), "v"(t));
                *dst = t;
                compiler_fence();
            }
            __syncthreads();
            uint32_t tcount[R];
            uint32_t tsum = 0;
            if (tid < DT) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t dg = tid * R + r;
                    uint32_t run = 0;
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) {
                        const uint32_t c = s_whist[w * RADIX + dg];
                        s_whist[w * RADIX + dg] = run;
                        run += c;
                    }
                    tcount[r] = run;
                    tsum += run;
                }
            }
            const uint32_t texcl = block_exclusive_sum<BLOCK>(tid < DT ? tsum : 0u, s_wsum);
            if (tid < DT) {
                uint32_t run = texcl;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t dg = tid * R + r;
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) s_whist[w * RADIX + dg] += run;
                    run += tcount[r];
                }
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                if (wave * WAVE_ITEMS + j * 64 >= n) continue;
                const uint32_t r = wh[__builtin_amdgcn_ubfe(key[j], shift, width)] + rnk[j];
                s_k[r] = key[j];
                if constexpr (VALS) s_v[r] = val[j];
            }
            __syncthreads();
            if (shift + BITS < static_cast<uint32_t>(key_bits)) {
#pragma unroll
                for (int j = 0; j < IPT; ++j) {
                    const uint32_t i = wslot0 + j * 64;
                    key[j] = i < n ? s_k[i] : ~0u;
                    if constexpr (VALS) val[j] = i < n ? s_v[i] : 0u;
                }
                // s_k is rewritten only after the next pass's first barrier
            }
        }
        uint32_t *out_k = to_temp ? d.tk : d.k;
        uint32_t *out_v = to_temp ? d.tv : d.v;
        for (uint32_t i = tid; i < n; i += BLOCK) {
            out_k[i] = s_k[i];
            if constexpr (VALS) out_v[i] = s_v[i];
        }
        __syncthreads();  // s_k and s_v are reused by the next segment
    }
}

// ---------------------------------------------------------------------------
// tiled segments: per-segment histograms and prefix sums
// ---------------------------------------------------------------------------

// Counts the digits of the passes in `digits` (bit p: digit p) per tiled
// segment into hist[row][p][d] (zeroed before; other rows stay zero).  Block
// b walks a contiguous range of tiles (tile_desc from k_seg_tilemap), so its
// counters stay in LDS across the tiles of one segment and
// are flushed to HBM (atomics) only when the segment changes.  Counting is
// as in k_histogram: C lane-class copies of the counters in padded LDS rows,
// and a wave batch whose keys share a pass's digit is counted with one add.
// The input of pass 0 is the segment's own arrays.
template <int BLOCK, int C>
__global__ __launch_bounds__(BLOCK) void k_seg_histogram(const SegDesc *__restrict__ tile_desc,
                                                         const SegHeader *__restrict__ h,
                                                         uint32_t *__restrict__ hist, uint32_t tile,
                                                         uint32_t digits) {
    constexpr int BINS = kSegPasses * kSegRadix;
    constexpr int ROW = BINS + 1;
    constexpr int WAVES = BLOCK / 64;
    constexpr int U = 16;
    constexpr uint32_t SPAN = 64 * U;  // keys per wave batch
    __shared__ uint32_t s_h[C * ROW];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    uint32_t *hc = s_h + (lane % C) * ROW;
    for (uint32_t i = tid; i < C * ROW; i += BLOCK) s_h[i] = 0u;
    const uint32_t total = h->total_tiles;
    const uint32_t per = (total + gridDim.x - 1) / gridDim.x;
    const uint32_t t_begin = min(total, blockIdx.x * per);
    const uint32_t t_end = min(total, t_begin + per);
    // adds the LDS counters into the segment's row and clears them
    auto flush = [&](uint32_t row) {
        __syncthreads();
        uint32_t *out = hist + static_cast<size_t>(row) * BINS;
        for (uint32_t i = tid; i < BINS; i += BLOCK) {
            uint32_t c = 0;
#pragma unroll
            for (int w = 0; w < C; ++w) {
                c += s_h[w * ROW + i];
                s_h[w * ROW + i] = 0u;
            }
            if (c) atomicAdd(&out[i], c);
        }
        __syncthreads();
    };
    __syncthreads();
    uint32_t cur = ~0u;  // row of the segment whose counts are in LDS (uniform)
    for (uint32_t t = t_begin; t < t_end; ++t) {
        const SegDesc d = tile_desc[t];
        if (d.row != cur) {
            if (cur != ~0u) flush(cur);
            cur = d.row;
        }
        const uint32_t start = (t - d.pad) * tile;
        const uint32_t valid = min(tile, d.n - start);
        const uint32_t *src = d.k + start;
        for (uint32_t base = wave * SPAN; base < valid; base += WAVES * SPAN) {
            uint32_t k[U];
            if (base + SPAN <= valid) {
#pragma unroll
                for (int u = 0; u < U; ++u) k[u] = src[base + u * 64 + lane];
                const uint32_t k0 = __builtin_amdgcn_readfirstlane(k[0]);
                uint32_t differ = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) differ |= k[u] ^ k0;
#pragma unroll
                for (int p = 0; p < kSegPasses; ++p) {
                    if (!((digits >> p) & 1u)) continue;
                    uint32_t *hp = hc + p * kSegRadix;
                    if (__builtin_amdgcn_ballot_w64(__builtin_amdgcn_ubfe(differ, p * kSegBits, kSegBits) != 0u) == 0u) {
                        if (lane == 0) atomicAdd(&hp[__builtin_amdgcn_ubfe(k0, p * kSegBits, kSegBits)], SPAN);
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[__builtin_amdgcn_ubfe(k[u], p * kSegBits, kSegBits)], 1u);
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t i = base + u * 64 + lane;
                    if (i >= valid) continue;
                    const uint32_t key = src[i];
#pragma unroll
                    for (int p = 0; p < kSegPasses; ++p)
                        if ((digits >> p) & 1u)
                            atomicAdd(&hc[p * kSegRadix + __builtin_amdgcn_ubfe(key, p * kSegBits, kSegBits)], 1u);
                }
            }
        }
    }
    if (cur != ~0u) flush(cur);
}

// base[row][p][d] = count of digits below d in pass p of the segment: one
// block of 256 threads per tiled segment at a time.
static __global__ __launch_bounds__(256) void k_seg_plan(const SegDesc *__restrict__ descs,
                                                  const uint32_t *__restrict__ list,
                                                  const SegHeader *__restrict__ h,
                                                  const uint32_t *__restrict__ hist, uint32_t *__restrict__ base) {
    __shared__ uint32_t s_wsum[4];
    const uint32_t count = h->count[kSegLarge];
    for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
        const size_t row = static_cast<size_t>(descs[list[e]].row) * kSegPasses * kSegRadix;
        for (int p = 0; p < kSegPasses; ++p) {
            const uint32_t c = hist[row + p * kSegRadix + threadIdx.x];
            base[row + p * kSegRadix + threadIdx.x] = block_exclusive_sum<256>(c, s_wsum);
            __syncthreads();  // s_wsum is reused
        }
    }
}

// ---------------------------------------------------------------------------
// tiled segments: one counting-sort pass over every listed segment
// ---------------------------------------------------------------------------

// One block per tile (of BLOCK * IPT items: the tile the tile map was built
// for), claimed as in k_onesweep from nchunks chunks of whole segments
// (chunk_counter: the launch's kChunks counters, zeroed before it; chunk
// bounds from k_seg_tilemap with the same nchunks), then the pass body of
// onesweep_tile on it; the tile's segment and first tile come from
// tile_desc.  The tile's segment runs pass `pass` (or its own d.pass when
// pass < 0) on digit digit0 + pass: even passes read k/v and write tk/tv,
// odd passes the reverse, so four passes leave the result in k/v and three
// in tk/tv.  The segment's lookback chain starts at its first tile.  Status words: one per
// tile and digit, zeroed before the launch.  PERSIST: a block claims tiles
// until none is left, so a grid of one block per CU covers any tile count
// (for calls whose tiled list is usually short or empty: the full grid's
// blocks would mostly start only to find nothing to do).
template <int BLOCK, int IPT, bool VALS, typename S, bool PERSIST = false>
__global__ __launch_bounds__(BLOCK) void k_seg_onesweep(const SegDesc *__restrict__ tile_desc,
                                                        const SegHeader *__restrict__ h, int pass,
                                                        const uint32_t *__restrict__ base, S *__restrict__ status,
                                                        uint32_t *__restrict__ chunk_counter,
                                                        uint32_t *__restrict__ error_flag, uint32_t nchunks,
                                                        uint32_t digit0) {
    constexpr int TILE = BLOCK * IPT;
    constexpr bool SMALL = sizeof(S) == 4;  // every segment below 2^30 items
    __shared__ OnesweepLds<kSegBits, BLOCK, IPT, uint32_t, uint32_t, VALS> lds;

    for (;;) {
        for (uint32_t i = threadIdx.x & 63u; i < static_cast<uint32_t>(kSegRadix); i += 64)
            lds.whist[(threadIdx.x >> 6) * kSegRadix + i] = 0u;
        if (threadIdx.x == 0) {
            uint32_t x = 0;
            lds.claim[0] = claim_chunked(h->chunk_start, nchunks, chunk_counter, x);
        }
        __syncthreads();
        const uint32_t tile = lds.claim[0];
        if (tile >= h->total_tiles) return;  // kNoTile too
        const SegDesc d = tile_desc[tile];
        const uint32_t first = d.pad;
        const uint32_t p = pass >= 0 ? static_cast<uint32_t>(pass) : d.pass;
        TileJob<uint32_t, uint32_t> job;
        job.src_k = (p & 1u) ? d.tk : d.k;
        job.src_v = (p & 1u) ? d.tv : d.v;
        job.dst_k = (p & 1u) ? d.k : d.tk;
        job.dst_v = (p & 1u) ? d.v : d.tv;
        const uint32_t dg = digit0 + p;
        job.base = base + (static_cast<size_t>(d.row) * kSegPasses + dg) * kSegRadix;
        job.item0 = static_cast<size_t>(tile - first) * TILE;
        job.shift = dg * kSegBits;
        job.width = kSegBits;
        job.tile = tile;
        job.first = first;
        job.valid = min(static_cast<uint32_t>(TILE), d.n - (tile - first) * static_cast<uint32_t>(TILE));
        job.bound = d.n;
        onesweep_tile<kSegBits, BLOCK, IPT, uint32_t, uint32_t, VALS, false, S, true, SMALL>(job, lds, status,
                                                                                            error_flag);
        if constexpr (!PERSIST) return;
        __syncthreads();  // the tile is out of the LDS before the next claim
    }
}

// ---------------------------------------------------------------------------
// a second MSD level: sub-bucket bounds from the buckets' digit counts
// ---------------------------------------------------------------------------

// One block of 256 threads per bucket b = [off[b], off[b + 1]) of a
// segmented call whose tiled list holds every bucket of two or more items
// (no whole-in-LDS classes) and whose histogram counted digit `digit`:
// sub[b * 256 + d] = off[b] + the bucket's items with a lower digit, so
// sub-bucket b * 256 + d holds the bucket's items of digit d once the call's
// pass on that digit has run.  A bucket of fewer than two items has no row:
// its sub-buckets are empty but the last, which holds it.  sub[256 *
// buckets] = off[buckets].
// Block 0 also copies the call's error word to *err (the next segmented
// call reuses the header).
static __global__ __launch_bounds__(256) void k_msd_subbuckets(const uint32_t *__restrict__ off,
                                                               const SegDesc *__restrict__ descs,
                                                               const uint32_t *__restrict__ hist, uint32_t digit,
                                                               uint32_t buckets, uint32_t *__restrict__ sub,
                                                               const SegHeader *__restrict__ h,
                                                               uint32_t *__restrict__ err) {
    __shared__ uint32_t s_wsum[4];
    const uint32_t b = blockIdx.x, d = threadIdx.x;
    const uint32_t a = off[b], e = off[b + 1];
    uint32_t c = 0;
    if (e - a >= 2u) c = hist[(static_cast<size_t>(descs[b].row) * kSegPasses + digit) * kSegRadix + d];
    const uint32_t below = block_exclusive_sum<256>(c, s_wsum);
    sub[static_cast<size_t>(b) * kSegRadix + d] = a + below;
    if (b + 1 == buckets && d == 0) sub[static_cast<size_t>(buckets) * kSegRadix] = e;
    if (b == 0 && d == 0) *err = h->error;
}

}  // namespace rt
