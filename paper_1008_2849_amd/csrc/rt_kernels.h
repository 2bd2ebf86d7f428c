// rt_kernels.h -- gfx950 kernels of the stable LSD radix sort.
//
// One sort is: an upfront read of the keys that builds the digit histograms
// of every pass at once; a planning kernel that turns them into each digit's
// first output slot (exclusive prefix sum), marks passes whose digit is
// constant as skipped and picks source/destination buffers on the device;
// then one "onesweep" kernel per executed pass.  Each onesweep block takes
// the next tile of the pass input, ranks its items stably with wave64
// ballots, publishes its per-digit counts, learns from the tiles before it
// (decoupled lookback) where each of its digit runs starts, gathers the tile
// by digit in LDS and writes every digit run to HBM as one burst of
// consecutive addresses.
//
// The counting-sort pass is the naive algorithm of Section 3 of Wassenberg &
// Sanders (histogram, exclusive prefix sum, scatter with increment); the pass
// order and stability requirement are Section 4's LSD radix sort.  The LDS
// staging plays the part of Section 2's software write-combining buffers:
// output leaves the chip in runs of consecutive addresses instead of one
// scattered word per item, and the tiles are large (16K items) so that a
// digit's run is 256 bytes long on average for uniform keys.
#include "rt_internal.h"

namespace rt {

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

// Lanes of the wave holding the same BITS-bit digit as this lane: one ballot
// per digit bit, keeping the lanes that agree with this lane on that bit.
// The whole wave must be active.  Per bit: the bit sign-extended to 0 or ~0,
// its ballot, and one three-input logic op per mask half.
template <int BITS>
__device__ __forceinline__ void match_digit(uint32_t d, uint32_t &lo, uint32_t &hi) {
    int s[BITS];
    uint64_t set[BITS];
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        s[b] = __builtin_amdgcn_sbfe(static_cast<int>(d), b, 1);  // 0 or -1
        // Keep s opaque so the ballot compares it directly instead of
        // re-deriving the bit with extra shifts.
        asm volatile("" : "+v"(s[b]));
    }
#pragma unroll
    for (int b = 0; b < BITS; ++b) set[b] = __builtin_amdgcn_ballot_w64(s[b] != 0);
    lo = ~0u;
    hi = ~0u;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        // 0x90 = a & ~(b ^ c): keep the lanes whose bit b equals ours
        lo = __builtin_amdgcn_bitop3_b32(lo, static_cast<uint32_t>(set[b]), static_cast<uint32_t>(s[b]), 0x90);
        hi = __builtin_amdgcn_bitop3_b32(hi, static_cast<uint32_t>(set[b] >> 32), static_cast<uint32_t>(s[b]),
                                         0x90);
    }
}

// Global-memory views: address space 1 lets the compiler use global (not
// flat) instructions, with a uniform 64-bit base and a 32-bit lane offset.
typedef __attribute__((address_space(1))) uint32_t g_u32;
typedef __attribute__((address_space(1))) char g_char;

// Element i of a global u32 array.  SMALL: i < 2^30, so the byte offset fits
// in 32 bits.
template <bool SMALL>
__device__ __forceinline__ const g_u32 *gelem(const uint32_t *base, size_t i) {
    // C-style casts: clang turns them into address-space casts
    if constexpr (SMALL)
        return (const g_u32 *)((const g_char *)base + static_cast<uint32_t>(i * 4u));
    else
        return (const g_u32 *)base + i;
}
template <bool SMALL>
__device__ __forceinline__ g_u32 *gelem(uint32_t *base, size_t i) {
    if constexpr (SMALL)
        return (g_u32 *)((g_char *)base + static_cast<uint32_t>(i * 4u));
    else
        return (g_u32 *)base + i;
}

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves (no LDS
// round trip): shifts by 1, 2, 4 and 8 lanes inside each row of 16, then
// row 0's total into row 1 and row 2's into row 3 (row_bcast:15), then the
// total of rows 0-1 into rows 2-3 (row_bcast:31).  A lane whose source lies
// outside its row adds the old value 0.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t x) {
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x111, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x112, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x114, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x118, 0xf, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x142, 0xa, 0xf, false));
    x += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x143, 0xc, 0xf, false));
    return x;
}

// Exclusive prefix sum of v over the block; every thread must call it.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *s_wsum) {
    constexpr int WAVES = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t x = wave_inclusive_sum(v);
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w)
        if (w < wave) before += s_wsum[w];
    return before + x - v;
}

// Sleep roughly `rounds` * 64 clocks (s_sleep takes an immediate).
__device__ __forceinline__ void backoff(uint32_t rounds) {
    for (uint32_t i = 0; i < rounds; ++i) __builtin_amdgcn_s_sleep(1);
}

// ---------------------------------------------------------------------------
// lookback status words: two flag bits over the running count.  32-bit
// words hold counts < 2^30; larger sorts use 64-bit words.
// ---------------------------------------------------------------------------

template <typename S>
struct Status;

template <>
struct Status<uint32_t> {
    __device__ static uint32_t make(uint32_t flag, uint32_t count) { return (flag << 30) | count; }
    __device__ static uint32_t flag(uint32_t s) { return s >> 30; }
    __device__ static uint32_t count(uint32_t s) { return s & 0x3FFFFFFFu; }
};

template <>
struct Status<uint64_t> {
    __device__ static uint64_t make(uint32_t flag, uint32_t count) {
        return (static_cast<uint64_t>(flag) << 62) | count;
    }
    __device__ static uint32_t flag(uint64_t s) { return static_cast<uint32_t>(s >> 62); }
    __device__ static uint32_t count(uint64_t s) { return static_cast<uint32_t>(s); }
};

constexpr uint32_t kFlagAgg = 1u;   // count of this tile alone
constexpr uint32_t kFlagIncl = 2u;  // count of this tile and all earlier ones

template <typename S>
__device__ __forceinline__ S status_load(const S *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
__device__ __forceinline__ void status_store(S *p, S v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

static __global__ __launch_bounds__(256) void k_fill_zero(uint32_t *__restrict__ p, size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < words; i += stride)
        p[i] = 0u;
}

static __global__ __launch_bounds__(64) void k_set_word(uint32_t *__restrict__ p, uint32_t v) {
    if (threadIdx.x == 0) *p = v;
}

// ---------------------------------------------------------------------------
// upfront histograms of all passes (one read of the keys)
// ---------------------------------------------------------------------------

struct HistArgs {
    uint32_t num_passes;
    uint32_t shift[kMaxPasses];
    uint32_t mask[kMaxPasses];
    uint32_t lds_offset[kMaxPasses];
    uint32_t total_bins;
    // per-chunk counts (CHUNKED): pass 0 by position, chunk x = keys
    // [pos_bound[x], pos_bound[x + 1]); pass p > 0 by the top bits of digit
    // p - 1, chunk = digit(p - 1) >> cshift[p - 1]
    uint32_t cshift[kMaxPasses];
    uint32_t pos_bound[kChunks + 1];
};

// Chunk of pass 0 that holds key i.
__device__ __forceinline__ uint32_t pos_chunk(const HistArgs &ha, size_t i) {
    uint32_t x = 0;
#pragma unroll
    for (int q = 1; q < kChunks; ++q) x += i >= ha.pos_bound[q] ? 1u : 0u;
    return x;
}

// Counts per pass and digit into hist[p * kMaxRadix + d], which must start at
// zero.  A block keeps C copies of the counters of all passes in LDS, one
// per lane class (lane mod C), in rows of total_bins + 1 words: lanes that
// hit the same digit then add into C different words in C different banks,
// so skewed keys no longer serialise on one LDS address.  Before counting a
// wave's batch of 64 * U keys, one test per pass checks whether the whole
// batch shares that pass's digit (constant bytes, runs of equal keys); such
// a digit is counted with a single add.  Keys are read in 256-byte slots.
//
// CHUNKED: every pass's counts are split by chunk (see PassPlan) into
// hist[(p * kChunks + x) * kChunkRadix + d], LDS rows kChunks times longer.
// The chunks of pass p > 0 are ranges of digit p - 1, which is how pass p's
// input (pass p - 1's output) is ordered, so one read of the keys gives
// every pass's per-chunk counts.  A wave's batch never straddles a chunk of
// pass 0 (the bounds are multiples of 1024 keys).
template <int BLOCK, int C, bool CHUNKED>
__device__ __forceinline__ void histogram_body(const uint32_t *__restrict__ keys, uint32_t n, const HistArgs &ha,
                                               uint32_t *__restrict__ hist, uint32_t *s_h) {
    constexpr int WAVES = BLOCK / 64;
    constexpr int U = 16;  // slots in flight per lane (8 measured 18 % slower on 2^28 keys)
    // s_h: C rows of total_bins + 1 counters
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t row = ha.total_bins + 1u;
    for (uint32_t i = tid; i < C * row; i += BLOCK) s_h[i] = 0u;
    __syncthreads();
    uint32_t *h = s_h + (lane % C) * row;

    const size_t wave_span = static_cast<size_t>(64) * U;
    const size_t stride = static_cast<size_t>(gridDim.x) * WAVES * wave_span;
    for (size_t base = (static_cast<size_t>(blockIdx.x) * WAVES + wave) * wave_span; base < n; base += stride) {
        uint32_t k[U];
        if (base + wave_span <= n) {
#pragma unroll
            for (int u = 0; u < U; ++u) k[u] = keys[base + u * 64 + lane];
            // bits in which some key of the batch differs from lane 0's first
            const uint32_t k0 = __builtin_amdgcn_readfirstlane(k[0]);
            uint32_t differ = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) differ |= k[u] ^ k0;
#pragma unroll
            for (int p = 0; p < kMaxPasses; ++p) {
                if (p >= static_cast<int>(ha.num_passes)) break;
                uint32_t *hp = h + ha.lds_offset[p];
                const uint32_t sh = ha.shift[p], m = ha.mask[p];
                if constexpr (!CHUNKED) {
                    if (__builtin_amdgcn_ballot_w64(((differ >> sh) & m) != 0u) == 0u) {
                        if (lane == 0) atomicAdd(&hp[(k0 >> sh) & m], static_cast<uint32_t>(64 * U));
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[(k[u] >> sh) & m], 1u);
                    }
                } else if (p == 0) {
                    hp += pos_chunk(ha, base) * (m + 1u);
                    if (__builtin_amdgcn_ballot_w64(((differ >> sh) & m) != 0u) == 0u) {
                        if (lane == 0) atomicAdd(&hp[(k0 >> sh) & m], static_cast<uint32_t>(64 * U));
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[(k[u] >> sh) & m], 1u);
                    }
                } else {
                    const uint32_t cs = ha.shift[p - 1] + ha.cshift[p - 1];
                    const uint32_t cm = ha.mask[p - 1] >> ha.cshift[p - 1];
                    const uint32_t w = 32u - __builtin_clz(m);
                    if (__builtin_amdgcn_ballot_w64((differ & ((m << sh) | (cm << cs))) != 0u) == 0u) {
                        if (lane == 0)
                            atomicAdd(&hp[(((k0 >> cs) & cm) << w) | ((k0 >> sh) & m)], static_cast<uint32_t>(64 * U));
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[(((k[u] >> cs) & cm) << w) | ((k[u] >> sh) & m)], 1u);
                    }
                }
            }
        } else {  // the ragged end of the array
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = base + u * 64 + lane;
                if (i >= n) continue;
                const uint32_t key = keys[i];
                for (int p = 0; p < static_cast<int>(ha.num_passes); ++p) {
                    uint32_t bin = (key >> ha.shift[p]) & ha.mask[p];
                    if constexpr (CHUNKED) {
                        const uint32_t w = 32u - __builtin_clz(ha.mask[p]);
                        const uint32_t x = p == 0 ? pos_chunk(ha, i)
                                                  : ((key >> ha.shift[p - 1]) & ha.mask[p - 1]) >> ha.cshift[p - 1];
                        bin |= x << w;
                    }
                    atomicAdd(&h[ha.lds_offset[p] + bin], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < ha.total_bins; i += BLOCK) {
        uint32_t c = 0;
#pragma unroll
        for (int w = 0; w < C; ++w) c += s_h[w * row + i];
        if (c == 0) continue;
        uint32_t p = 0;
        while (p + 1 < ha.num_passes && i >= ha.lds_offset[p + 1]) ++p;
        const uint32_t local = i - ha.lds_offset[p];
        if constexpr (CHUNKED) {
            const uint32_t w = 32u - __builtin_clz(ha.mask[p]);
            atomicAdd(&hist[(p * kChunks + (local >> w)) * kChunkRadix + (local & ha.mask[p])], c);
        } else {
            atomicAdd(&hist[p * kMaxRadix + local], c);
        }
    }
}

template <int BLOCK, int C, bool CHUNKED = false>
__global__ __launch_bounds__(BLOCK) void k_histogram(const uint32_t *__restrict__ keys, uint32_t n,
                                                     HistArgs ha, uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t s_h[];
    histogram_body<BLOCK, C, CHUNKED>(keys, n, ha, hist, s_h);
}

// The histogram of a sort that may count per chunk: per chunk (CC copies,
// args hc) if the probe chose it (*mode != 0), else plain (CP copies, hp).
template <int BLOCK, int CP, int CC>
__global__ __launch_bounds__(BLOCK) void k_histogram_auto(const uint32_t *__restrict__ keys, uint32_t n,
                                                          HistArgs hp, HistArgs hc, const uint32_t *__restrict__ mode,
                                                          uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t s_h[];
    if (*mode != 0u)
        histogram_body<BLOCK, CC, true>(keys, n, hc, hist, s_h);
    else
        histogram_body<BLOCK, CP, false>(keys, n, hp, hist, s_h);
}

// Chooses, for one sort, between per-chunk counts with one lookback chain
// per chunk (*mode = 1) and plain counts with one chain per pass (*mode =
// 0), from kProbeSamples keys in evenly spaced runs.  Per-chunk counts leave
// room for only two LDS copies per histogram block, so a frequent (chunk,
// digit) bin serialises its atomics; and when one chunk of pass p > 0 (a
// range of digit p - 1) holds most items, its tiles are claimed by every XCD
// in turn and the pass gains nothing.  Either is a reason for one chain: a bin above 1/64 of
// the samples (unless the pass's digit is constant: batches of equal digits
// are counted with one add), or a chunk above 1/4 (unless digit p - 1 is
// constant: then the pass has a single chunk and loses nothing).
constexpr uint32_t kProbeSamples = 8192;  // 128 runs of 64 consecutive keys

template <typename T, typename F>
__device__ __forceinline__ T wave_reduce(T v, F op) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    return v;
}

template <int BLOCK, typename K = uint32_t>
__global__ __launch_bounds__(BLOCK) void k_chunk_probe(const K *__restrict__ keys, uint32_t n, HistArgs ha,
                                                       uint32_t *__restrict__ mode) {
    constexpr int WAVES = BLOCK / 64;
    constexpr int RUNS = static_cast<int>(kProbeSamples / 64);
    constexpr int PER = RUNS / WAVES;  // runs per wave = keys per lane
    __shared__ uint32_t s_tab[kChunks * kChunkRadix];
    __shared__ uint32_t s_chunk[kChunks];
    __shared__ uint32_t s_lo[kMaxPasses], s_hi[kMaxPasses];
    __shared__ uint32_t s_max, s_bad;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    // runs of consecutive keys: a few hundred pages touched, not thousands
    K k[PER];  // 32- or 64-bit keys
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint64_t start = static_cast<uint64_t>(wave * PER + j) * n / RUNS;
        k[j] = keys[min(start + lane, static_cast<uint64_t>(n) - 1u)];
    }
    if (tid < kMaxPasses) {
        s_lo[tid] = ~0u;
        s_hi[tid] = 0u;
    }
    if (tid == 0) s_bad = 0u;
    __syncthreads();
    for (uint32_t p = 0; p < ha.num_passes; ++p) {
        uint32_t lo = ~0u, hi = 0u;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t d = static_cast<uint32_t>(k[j] >> ha.shift[p]) & ha.mask[p];
            lo = min(lo, d);
            hi = max(hi, d);
        }
        lo = wave_reduce(lo, [](uint32_t x, uint32_t y) { return min(x, y); });
        hi = wave_reduce(hi, [](uint32_t x, uint32_t y) { return max(x, y); });
        if (lane == 0) {
            atomicMin(&s_lo[p], lo);
            atomicMax(&s_hi[p], hi);
        }
    }
    for (uint32_t p = 0; p < ha.num_passes; ++p) {
        for (uint32_t i = tid; i < kChunks * kChunkRadix; i += BLOCK) s_tab[i] = 0u;
        if (tid < kChunks) s_chunk[tid] = 0u;
        if (tid == 0) s_max = 0u;
        __syncthreads();
        const uint32_t w = 32u - __builtin_clz(ha.mask[p]);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t x = p == 0 ? 0u : (static_cast<uint32_t>(k[j] >> ha.shift[p - 1]) & ha.mask[p - 1]) >> ha.cshift[p - 1];
            atomicAdd(&s_tab[(x << w) | (static_cast<uint32_t>(k[j] >> ha.shift[p]) & ha.mask[p])], 1u);
        }
        __syncthreads();
        uint32_t m = 0;
        for (uint32_t i = tid; i < (static_cast<uint32_t>(kChunks) << w); i += BLOCK) {
            const uint32_t c = s_tab[i];
            m = max(m, c);
            if (w >= 6u) {  // a wave's 64 entries share a chunk: one add per wave
                const uint32_t t = wave_reduce(c, [](uint32_t x, uint32_t y) { return x + y; });
                if (lane == 0) atomicAdd(&s_chunk[i >> w], t);
            } else if (c != 0u) {
                atomicAdd(&s_chunk[i >> w], c);
            }
        }
        m = wave_reduce(m, [](uint32_t x, uint32_t y) { return max(x, y); });
        if (lane == 0) atomicMax(&s_max, m);
        __syncthreads();
        if (tid == 0) {
            if (s_lo[p] != s_hi[p] && s_max > kProbeSamples / 64) s_bad = 1u;
            if (p > 0 && s_lo[p - 1] != s_hi[p - 1]) {
                uint32_t mc = 0;
                for (int x = 0; x < kChunks; ++x) mc = max(mc, s_chunk[x]);
                if (mc > kProbeSamples / 4) s_bad = 1u;
            }
        }
        __syncthreads();
    }
    if (tid == 0) *mode = s_bad ? 0u : 1u;
}

// ---------------------------------------------------------------------------
// planning: exclusive prefix sums, pass skipping, buffer assignment
// ---------------------------------------------------------------------------

// The chunk fields of pass p's plan (see k_plan), written in place.
// prev_start[x]: where chunk x's first digit of pass p - 1 starts.
__device__ inline void plan_chunks(const PlanArgs &a, bool chunked, const uint32_t *prev_start,
                                   const uint32_t *base, uint32_t p, PassPlan *pp) {
    if (!pp->active) return;  // the pass kernel returns before reading them
    uint32_t cs[kChunks + 1];
#pragma unroll
    for (int x = 0; x <= kChunks; ++x) cs[x] = a.n;
    cs[0] = 0u;
    pp->nchunks = 1;
    pp->cbase = base + p * kMaxRadix;
    if (a.chunk_ctr != nullptr && a.tile != 0u && chunked) {
        pp->nchunks = kChunks;
        pp->cbase = a.cbase + p * kChunks * kChunkRadix;
        if (p == 0) {
#pragma unroll
            for (int x = 1; x < kChunks; ++x) cs[x] = min(a.pos_bound[x], a.n);
        } else {
            const uint32_t w = a.width[p - 1];
            const uint32_t nch = 1u << (w > 3u ? 3u : w);
#pragma unroll
            for (uint32_t x = 1; x < kChunks; ++x)
                if (x < nch) cs[x] = prev_start[x];
        }
    }
    uint32_t t = 0;
#pragma unroll
    for (int x = 0; x < kChunks; ++x) {
        pp->cstart[x] = cs[x];
        pp->ctile[x] = t;
        if (a.tile != 0u && cs[x + 1] > cs[x])  // tiles of the global grid that meet [cs[x], cs[x + 1])
            t += (cs[x + 1] - 1u) / a.tile + 1u - cs[x] / a.tile;
    }
    pp->cstart[kChunks] = a.n;
    pp->ctile[kChunks] = t;
}

// One block of 256 threads; thread t covers bins [8t, 8t + 8) of a pass.
// Also clears the tile counters of the passes and the error word after them.
//
// Chunks (a.chunk_ctr set): with a.chunked the histograms are per chunk (see
// k_histogram) and every pass gets kChunks chunks: pass 0 by position, pass
// p > 0 by the top bits of digit p - 1, so that chunk x of pass p starts
// where digit x << cshift starts in pass p - 1's output.  (If pass p - 1 is
// skipped its digit is constant, its output order is its input order and
// all items fall in one chunk, so the rule holds for skipped passes too.)
// Chunk x's output slot of digit d is the digit's start plus the counts of
// d in chunks 0..x-1.  Without a.chunked every pass is one chunk.
static __global__ __launch_bounds__(256) void k_plan(PlanArgs a, const uint32_t *__restrict__ hist,
                                              uint32_t *__restrict__ base, SortPlan *__restrict__ plan,
                                              uint32_t *__restrict__ tile_counters, uint32_t direct) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_constant[kMaxPasses];
    __shared__ uint32_t s_cstart[kMaxPasses + 1][kChunks];  // [p][x]: base of pass p - 1 at chunk x's first digit
    const uint32_t tid = threadIdx.x;
    // the histograms are per chunk only if the sort allows it and the probe
    // chose it (see k_chunk_probe)
    const bool chunked = a.chunked && (a.mode == nullptr || *a.mode != 0u);
    if (tid < kMaxPasses) {
        s_constant[tid] = 0u;
        tile_counters[tid] = 0u;
    }
    if (tid == kMaxPasses) tile_counters[kMaxPasses] = 0u;  // the error word
    if (a.chunk_ctr != nullptr)
        for (uint32_t i = tid; i < kMaxPasses * kChunks; i += 256) a.chunk_ctr[i] = 0u;
    __syncthreads();
    for (uint32_t p = 0; p < a.num_passes; ++p) {
        const uint32_t bins = 1u << a.width[p];
        if (chunked) {
            // digits of at most 8 bits: thread t owns digit t, its chunk
            // counts loaded together
            const uint32_t d = tid;
            uint32_t h[kChunks];
            uint32_t c = 0;
#pragma unroll
            for (int x = 0; x < kChunks; ++x) {
                h[x] = d < bins ? hist[(p * kChunks + x) * kChunkRadix + d] : 0u;
                c += h[x];
            }
            if (c == a.n) s_constant[p] = 1u;  // every key has this digit
            const uint32_t run = block_exclusive_sum<256>(c, s_wsum);
            base[p * kMaxRadix + d] = d < bins ? run : a.n;
            for (uint32_t i = d + 256; i < static_cast<uint32_t>(kMaxRadix); i += 256) base[p * kMaxRadix + i] = a.n;
            if (d < bins) {
                uint32_t r = run;
#pragma unroll
                for (int x = 0; x < kChunks; ++x) {
                    a.cbase[(p * kChunks + x) * kChunkRadix + d] = r;
                    r += h[x];
                }
                // pass p + 1's chunk x starts where digit x << cshift of this pass starts
                const uint32_t cshift = a.width[p] > 3u ? a.width[p] - 3u : 0u;
                if ((d & ((1u << cshift) - 1u)) == 0u && (d >> cshift) < kChunks) s_cstart[p + 1][d >> cshift] = run;
            }
            __syncthreads();  // s_wsum is reused by the next pass; s_cstart is read below
            continue;
        }
        uint32_t c[8];
        uint32_t sum = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint32_t d = tid * 8 + i;
            c[i] = d < bins ? hist[p * kMaxRadix + d] : 0u;
            sum += c[i];
            if (c[i] == a.n) s_constant[p] = 1u;  // every key has this digit
        }
        uint32_t run = block_exclusive_sum<256>(sum, s_wsum);
#pragma unroll
        for (int i = 0; i < 8; ++i) {  // bins past the digit's range start at n
            base[p * kMaxRadix + tid * 8 + i] = run;
            run += c[i];
        }
        __syncthreads();  // s_wsum is reused by the next pass
    }
    if (tid != 0) return;

    uint32_t active[kMaxPasses];
    uint32_t executed = 0;
    for (uint32_t p = 0; p < kMaxPasses; ++p) {
        active[p] = p < a.num_passes && (direct || a.no_skip || !s_constant[p]);
        executed += active[p];
    }
    // Buffers: U = caller's arrays, A/B = temporaries.  The last executed pass
    // must write U: an even count alternates U->A->U...; an odd count >= 3
    // starts U->A->B->U and then alternates; a single pass goes U->A and is
    // copied back.  `direct` (one explicit pass) reads U and writes A.
    const uint32_t *src_k = a.user_k, *src_v = a.user_v;
    uint32_t j = 0;
    for (uint32_t p = 0; p < kMaxPasses; ++p) {
        PassPlan pp;
        pp.active = active[p];
        pp.shift = a.shift[p];
        pp.width = a.width[p];
        pp.pad[0] = pp.pad[1] = 0;
        pp.src_k = src_k;
        pp.src_v = src_v;
        pp.dst_k = nullptr;
        pp.dst_v = nullptr;
        if (active[p]) {
            uint32_t *dk, *dv;
            if (direct) {
                dk = a.t1_k; dv = a.t1_v;
            } else if (executed == 1) {
                dk = a.t1_k; dv = a.t1_v;
            } else if ((executed & 1u) && j < 3) {
                dk = j == 0 ? a.t1_k : (j == 1 ? a.t2_k : a.user_k);
                dv = j == 0 ? a.t1_v : (j == 1 ? a.t2_v : a.user_v);
            } else {
                const uint32_t k = (executed & 1u) ? j - 3 : j;  // position in the alternation
                dk = (k & 1u) ? a.user_k : a.t1_k;
                dv = (k & 1u) ? a.user_v : a.t1_v;
            }
            pp.dst_k = dk;
            pp.dst_v = dv;
            src_k = dk;
            src_v = dv;
            ++j;
        }
        plan->pass[p] = pp;
        plan_chunks(a, chunked, s_cstart[p], base, p, &plan->pass[p]);  // in place: no indexed local copy
    }
    plan->executed = executed;
    plan->copy_back = (!direct && executed == 1) ? 1u : 0u;
}

// Fused next-digit histogram (RT_FLAG_FUSED_HISTOGRAM): a pass counts the
// next pass's digit (at most 8 bits) of the items it writes into
// kFusedCopies copies of that pass's histogram row, spread by block so that
// fewer blocks add into one word; copy c holds bins [c * 256, c * 256 + 256)
// of the row (the row has kMaxRadix words).
constexpr int kFusedBins = 256;
constexpr int kFusedCopies = kMaxRadix / kFusedBins;

// Pass `pass`'s digit starts from its fused histogram (RT_FLAG_FUSED_HISTOGRAM):
// the sum of the kFusedCopies copies of its row, then the exclusive prefix
// sum, written to its base row (digits past its range start at n).  One
// block of 256 threads, launched after pass - 1 (which counted the row).
// The sort runs on one chain, so the row is the pass's whole plan.
static __global__ __launch_bounds__(256) void k_plan_fused(const uint32_t *__restrict__ hist,
                                                    uint32_t *__restrict__ base, uint32_t pass, uint32_t width,
                                                    uint32_t n) {
    __shared__ uint32_t s_wsum[4];
    const uint32_t d = threadIdx.x;
    const uint32_t *row = hist + static_cast<size_t>(pass) * kMaxRadix;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kFusedCopies; ++k) c += row[k * kFusedBins + d];
    const uint32_t run = block_exclusive_sum<256>(c, s_wsum);
    uint32_t *out = base + static_cast<size_t>(pass) * kMaxRadix;
    out[d] = d < (1u << width) ? run : n;
    for (uint32_t i = d + 256; i < static_cast<uint32_t>(kMaxRadix); i += 256) out[i] = n;
}

// ---------------------------------------------------------------------------
// onesweep counting-sort pass
// ---------------------------------------------------------------------------

// Decoupled lookback for one digit of one tile: the sum of that digit's
// counts over all earlier tiles.  Earlier tiles publish an aggregate (their
// own count) and later an inclusive prefix; the walk goes back from the
// previous tile, adding aggregates, until it reaches an inclusive prefix.
// The status words of kLookbackBatch earlier tiles are loaded at once.
//
// Every earlier tile publishes within microseconds of starting, and a tile
// only waits on tiles that were claimed (and so started) before it.  The
// wait is still bounded: after kLookbackSpinLimit fruitless polls the walk
// raises the error flag and stops, which leaves a wrong result rather than
// a GPU that never finishes.
constexpr int kLookbackBatch = 8;
constexpr uint32_t kLookbackSpinLimit = 1u << 22;
constexpr uint32_t kErrLookbackTimeout = 1u;

//
// The chain starts at tile lo (the first tile of a chunk or segment): only
// tiles [lo, tile) are summed.
template <typename S>
__device__ __forceinline__ uint32_t lookback_digit(const S *__restrict__ status, int32_t tile, int32_t lo,
                                                   uint32_t digit, int radix, uint32_t *__restrict__ error_flag) {
    using St = Status<S>;
    uint32_t excl = 0;
    int32_t at = tile - 1;  // the nearest tile not yet accounted for
    uint32_t idle = 0, nap = 1;
    while (at >= lo) {
        S w[kLookbackBatch];
#pragma unroll
        for (int b = 0; b < kLookbackBatch; ++b)
            w[b] = (at - b >= lo) ? status_load(status + static_cast<size_t>(at - b) * radix + digit) : S(0);
        bool finished = false, stalled = false;
        int32_t consumed = 0;
#pragma unroll
        for (int b = 0; b < kLookbackBatch; ++b) {
            if (finished || stalled || at - b < lo) continue;
            const uint32_t f = St::flag(w[b]);
            if (f == 0u) {
                stalled = true;  // not published yet: resume from this tile
            } else {
                excl += St::count(w[b]);
                ++consumed;
                if (f == kFlagIncl) finished = true;
            }
        }
        if (finished) break;
        at -= consumed;
        if (stalled && consumed == 0) {
            backoff(nap);
            nap = nap < 16 ? nap * 2 : 16;
            if (++idle > kLookbackSpinLimit) {
                atomicOr(error_flag, kErrLookbackTimeout);
                break;
            }
        } else {
            nap = 1;
        }
    }
    return excl;
}

constexpr uint32_t kNoTile = 0xFFFFFFFFu;

// The XCD this wave runs on (0..7 on the MI355X).
__device__ __forceinline__ uint32_t xcd_id() {
    uint32_t x;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(x));
    return x;
}

// Claims an index for the block (called by one thread).  Chunk x owns the
// indices [bound[x], bound[x + 1]) and hands them out in order from its
// counter ctr[x]; the block tries the chunk of its own XCD first, then the
// next chunk with indices left.  Returns kNoTile once every chunk is
// exhausted.  Only the order within a chunk matters for progress: a block
// waits only on indices claimed before it, whichever XCD they run on.
__device__ __forceinline__ uint32_t claim_chunked(const uint32_t *__restrict__ bound, uint32_t nch,
                                                  uint32_t *__restrict__ ctr, uint32_t &chunk) {
    const uint32_t x0 = xcd_id() % nch;
    {
        // the atomic goes out with the loads of the chunk's bounds (one
        // round trip): a claim past the end of a chunk is simply dropped
        const uint32_t k = atomicAdd(ctr + x0, 1u);
        const uint32_t b0 = bound[x0], size = bound[x0 + 1] - b0;
        if (k < size) {
            chunk = x0;
            return b0 + k;
        }
    }
    if (nch == 1u) return kNoTile;
    // The own chunk is exhausted: read every counter at once rather than
    // spend one atomic (a memory round trip) per full chunk.  Counters only
    // grow, so a chunk seen full stays full.
    uint32_t full = 0;
#pragma unroll
    for (int y = 0; y < kChunks; ++y) {
        if (y >= static_cast<int>(nch)) break;
        const uint32_t used = __hip_atomic_load(ctr + y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (used >= bound[y + 1] - bound[y]) full |= 1u << y;
    }
    for (uint32_t q = 1; q < nch; ++q) {
        const uint32_t x = (x0 + q) % nch;
        if ((full >> x) & 1u) continue;
        const uint32_t k = atomicAdd(ctr + x, 1u);
        if (k < bound[x + 1] - bound[x]) {
            chunk = x;
            return bound[x] + k;
        }
    }
    return kNoTile;
}

// Claims a tile of a pass (one thread): its lookback index, the lookback
// index of its chunk's first tile, its chunk, its first input item and its
// item count; tile = kNoTile once every chunk is exhausted.  The chunk tables
// are read from the plan in global memory: indexing a by-value copy with a
// run-time chunk would put it in scratch memory.
template <int TILE>
__device__ __forceinline__ void claim_tile(const PassPlan *__restrict__ pp, uint32_t *chunk_counter, uint32_t &tile,
                                           uint32_t &first, uint32_t &chunk, uint32_t &lo, uint32_t &valid) {
    uint32_t x = 0;
    tile = claim_chunked(pp->ctile, pp->nchunks, chunk_counter, x);
    if (tile == kNoTile) return;
    const uint32_t t0 = pp->ctile[x];
    const uint32_t c0 = pp->cstart[x], c1 = pp->cstart[x + 1];
    const uint64_t g = c0 / TILE + (tile - t0);  // tile of the global grid
    const uint64_t b = max(static_cast<uint64_t>(c0), g * TILE);
    const uint64_t e = min(static_cast<uint64_t>(c1), (g + 1) * TILE);
    first = t0;
    chunk = x;
    lo = static_cast<uint32_t>(b);
    valid = static_cast<uint32_t>(e - b);
}

// ---------------------------------------------------------------------------
// the onesweep counting-sort pass over one tile: one body for 32-bit keys,
// 64-bit keys and segments
// ---------------------------------------------------------------------------

// Global view of element i of an array of T in address space 1 (global
// instructions with a uniform base).  SMALL: the byte offset i * sizeof(T)
// fits in 32 bits, so it is formed in 32-bit arithmetic.
template <typename T, bool SMALL>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const T *base, size_t i) {
    typedef const __attribute__((address_space(1))) T gt;
    if constexpr (SMALL)
        return (gt *)((const g_char *)base + static_cast<uint32_t>(i * sizeof(T)));
    else
        return (gt *)base + i;
}
template <typename T, bool SMALL>
__device__ __forceinline__ __attribute__((address_space(1))) T *gptr(T *base, size_t i) {
    typedef __attribute__((address_space(1))) T gt;
    if constexpr (SMALL)
        return (gt *)((g_char *)base + static_cast<uint32_t>(i * sizeof(T)));
    else
        return (gt *)base + i;
}

template <bool NT, typename T>
__device__ __forceinline__ void store_t(__attribute__((address_space(1))) T *p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// The pass's digit of a key: bits [shift, shift + width) (width <= 11).
__device__ __forceinline__ uint32_t key_digit(uint32_t key, uint32_t shift, uint32_t width) {
    return __builtin_amdgcn_ubfe(key, shift, width);
}
__device__ __forceinline__ uint32_t key_digit(uint64_t key, uint32_t shift, uint32_t width) {
    return static_cast<uint32_t>(key >> shift) & ((1u << width) - 1u);
}

// One tile of a counting-sort pass, as its kernel has claimed it.  Items
// are read from src at [item0, item0 + valid) and written to dst; base[d] is
// the output slot, in dst, of the first item of digit d that this tile's
// lookback chain (its XCD chunk, or its segment) holds.  Lookback index
// `tile` waits on the chain's tiles [first, tile).  Every store is clamped
// to [0, bound).
template <typename K, typename V>
struct TileJob {
    const K *src_k;
    const V *src_v;
    K *dst_k;
    V *dst_v;
    const uint32_t *base;
    size_t item0;
    uint32_t shift, width;
    uint32_t tile, first;
    uint32_t valid;
    uint32_t bound;
    // FUSED: where the next pass's digit counts go (its histogram row) and
    // that digit's bits
    uint32_t *next_hist;
    uint32_t next_shift, next_width;
};

// LDS of one onesweep block: the tile staged by digit, per-wave digit
// counters (then offsets) with a 64-word scratch row per wave that absorbs
// the counter writes of non-leader lanes, each digit's output slot, the
// block scan's wave sums, and the claimed tile (broadcast by thread 0).
template <int BITS, int BLOCK, int IPT, typename K, typename V, bool VALS, bool FUSED = false, bool SEQ = false>
struct OnesweepLds {
    static constexpr int RADIX = 1 << BITS;
    static constexpr int WAVES = BLOCK / 64;
    static constexpr int TILE = BLOCK * IPT;
    static_assert(!SEQ || (VALS && sizeof(V) <= sizeof(K)), "sequential staging puts the values in the key stage");
    K stage_k[TILE];
    V stage_v[(VALS && !SEQ) ? TILE : 1];
    uint32_t whist[WAVES * RADIX + WAVES * 64];
    uint32_t gbase[RADIX];
    uint32_t wsum[WAVES];
    uint32_t claim[6];
    uint32_t fused[FUSED ? kFusedBins : 1];  // the tile's counts of the next pass's digit
};

// Stable rank of a wave's items, slot by slot and lane by lane (input
// order): rnk[j] = the wave's count of the digit before slot j plus the
// lanes below with that digit, from 8-bit (or BITS-bit) ballot matching.
// The first lane of each digit advances the wave's counter; the others
// write their private scratch word, so no atomics are needed.  mbcnt and
// bcnt add the counter while they count.  A partial tile's empty slots take
// the last digit, so they rank behind every item.  With VALS and FULL the
// tile's values are loaded halfway through (after the keys, which the
// ranking waits on first).
template <int BITS, int IPT, typename K, typename V, bool VALS, bool SMALL, bool FULL>
__device__ __forceinline__ void rank_items(const K (&key)[IPT], V (&val)[VALS ? IPT : 1], uint32_t (&rnk)[IPT],
                                           uint32_t *wh, uint32_t *scratch, uint32_t shift, uint32_t width,
                                           uint32_t valid, uint32_t wslot0, const V *src_v, size_t item0) {
    constexpr uint32_t RADIX = 1u << BITS;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = key_digit(key[j], shift, width);
        if (!FULL && wslot0 + j * 64 >= valid) d = RADIX - 1;
        uint32_t lo, hi;
        match_digit<BITS>(d, lo, hi);
        const uint32_t cnt = wh[d];
        const uint32_t r = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, cnt));
        rnk[j] = r;
        uint32_t *dst = r == cnt ? wh + d : scratch;
        // popcount(lo) + popcount(hi) + cnt in two ops: v_bcnt adds its
        // second operand
        uint32_t t;
        asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(t) : "v"(lo), "v"(cnt));
        asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(t) : "v"(hi), "v"(t));
        *dst = t;
        compiler_fence();
        if constexpr (VALS && FULL) {
            if (j == IPT / 2 - 1) {
#pragma unroll
                for (int q = 0; q < IPT; ++q) val[q] = *gptr<V, SMALL>(src_v, item0 + wslot0 + q * 64);
            }
        }
    }
}

// One tile of a pass.  Wave w owns items [w * 64 * IPT, (w + 1) * 64 * IPT)
// of the tile and lane l holds item j * 64 + l of that range in slot j, so
// slot-by-slot, lane-by-lane processing follows input order (stability).
// Phases: load the keys (each slot of a wave is 64 consecutive items) ->
// rank every item inside its wave -> per-digit tile counts, published as
// the tile's aggregate -> tile-local digit offsets -> gather keys and
// values by digit in LDS -> lookback for the global offset of each digit ->
// write every digit run to consecutive output addresses.
//
// STAGE = false drops the gather: every item is written straight from its
// registers to its output slot, so a wave's stores scatter over the digit
// runs.  This is the pass without write-combining (the paper's "VM only"
// counterpart), kept to measure what the staging buys.
//
// SEQ stages the keys, scatters them, then stages and scatters the values
// through the same LDS: a tile whose keys and values would not fit the LDS
// together (16K items of 64-bit keys with 4- or 8-byte values) keeps its
// size at the cost of two more barriers.
template <int BITS, int BLOCK, int IPT, typename K, typename V, bool VALS, bool NT, typename S, bool STAGE,
          bool SMALL, bool FUSED = false, bool SEQ = false>
__device__ __forceinline__ void onesweep_tile(const TileJob<K, V> &job,
                                              OnesweepLds<BITS, BLOCK, IPT, K, V, VALS, FUSED, SEQ> &lds,
                                              S *__restrict__ status, uint32_t *__restrict__ error_flag) {
    constexpr int RADIX = 1 << BITS;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * IPT;
    constexpr int WAVE_ITEMS = 64 * IPT;
    constexpr int R = RADIX >= BLOCK ? RADIX / BLOCK : 1;  // digits per owning thread
    constexpr int DT = RADIX / R;                            // owning threads
    using St = Status<S>;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t shift = job.shift, width = job.width, valid = job.valid;
    const bool full = valid == static_cast<uint32_t>(TILE);
    const uint32_t wslot0 = wave * WAVE_ITEMS + lane;  // tile index of this lane's slot 0
    uint32_t *wh = lds.whist + wave * RADIX;
    uint32_t *scratch = lds.whist + WAVES * RADIX + wave * 64 + lane;

    // ---- load the keys (a partial tile: its values too)
    K key[IPT];
    V val[VALS ? IPT : 1];
    if (full) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) key[j] = *gptr<K, SMALL>(job.src_k, job.item0 + wslot0 + j * 64);
    } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j)
            key[j] = (wslot0 + j * 64 < valid) ? *gptr<K, SMALL>(job.src_k, job.item0 + wslot0 + j * 64) : K(0);
        if constexpr (VALS) {
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                val[j] = (wslot0 + j * 64 < valid) ? *gptr<V, SMALL>(job.src_v, job.item0 + wslot0 + j * 64) : V(0);
        }
    }

    // ---- stable rank inside the wave, per-wave digit counts in LDS
    uint32_t rnk[IPT];
    if (full)
        rank_items<BITS, IPT, K, V, VALS, SMALL, true>(key, val, rnk, wh, scratch, shift, width, valid, wslot0,
                                                      job.src_v, job.item0);
    else
        rank_items<BITS, IPT, K, V, VALS, SMALL, false>(key, val, rnk, wh, scratch, shift, width, valid, wslot0,
                                                       job.src_v, job.item0);
    __syncthreads();

    // ---- per digit: counts of earlier waves (kept in registers), the tile
    // count, published as the tile's aggregate (inclusive at once for a
    // chain's first tile); after the block scan each wave's counter becomes
    // the digit's LDS offset for that wave, written once
    uint32_t tcount[R];
    uint32_t wrun[R][WAVES];
    uint32_t tsum = 0;
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                wrun[r][w] = run;
                run += lds.whist[w * RADIX + d];
            }
            // a partial tile's empty slots ranked as the last digit: they
            // are not items (a chain's first tile can be partial and still
            // have successors that add this count)
            if (d == RADIX - 1) run -= TILE - valid;
            tcount[r] = run;
            tsum += run;
            status_store(status + static_cast<size_t>(job.tile) * RADIX + d,
                         St::make(job.tile == job.first ? kFlagIncl : kFlagAgg, run));
        }
    }
    const uint32_t texcl = block_exclusive_sum<BLOCK>(tid < DT ? tsum : 0u, lds.wsum);
    uint32_t dexcl[R];
    if (tid < DT) {
        uint32_t run = texcl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            dexcl[r] = run;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) lds.whist[w * RADIX + d] = wrun[r][w] + run;
            run += tcount[r];
        }
    }
    __syncthreads();

    // ---- gather keys and values by digit in LDS (tile rank = digit start +
    // earlier waves + rank inside the wave): the GPU form of software
    // write-combining, each digit's run now contiguous
    if constexpr (STAGE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            uint32_t d = key_digit(key[j], shift, width);
            if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
            const uint32_t r = wh[d] + rnk[j];
            lds.stage_k[r] = key[j];
            if constexpr (VALS && !SEQ) lds.stage_v[r] = val[j];
            if constexpr (SEQ) rnk[j] = r;  // the value's stage slot, after the keys have left
        }
    }

    // ---- lookback: the count of each digit in the chain's earlier tiles
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            const uint32_t excl = lookback_digit<S>(status, static_cast<int32_t>(job.tile),
                                                    static_cast<int32_t>(job.first), d, RADIX, error_flag);
            if (job.tile != job.first)
                status_store(status + static_cast<size_t>(job.tile) * RADIX + d, St::make(kFlagIncl, excl + tcount[r]));
            // LDS slot i of digit d goes to output slot gbase[d] + i
            lds.gbase[d] = job.base[d] + excl - dexcl[r];
        }
    }
    __syncthreads();

    // ---- scatter: consecutive LDS slots of one digit go to consecutive
    // output addresses.  The clamp costs one op and keeps a logic error from
    // ever turning into a store outside the array.  A full tile needs no
    // per-slot guard, so the LDS reads of all slots are issued together.
    const uint32_t last = job.bound - 1u;
    if constexpr (STAGE && SEQ) {
        static_assert(!FUSED && !NT, "sequential staging: plain stores, no fused counts");
        // keys first, keeping each slot's output position; then the values
        // through the same stage, to the same positions
        uint32_t sp[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = j * BLOCK + tid;
            const K k = lds.stage_k[i];
            sp[j] = min(lds.gbase[key_digit(k, shift, width)] + i, last);
            if (full || i < valid) store_t<NT, K>(gptr<K, SMALL>(job.dst_k, sp[j]), k);
        }
        __syncthreads();  // every key out of the stage
        V *stage_v = reinterpret_cast<V *>(lds.stage_k);
#pragma unroll
        for (int j = 0; j < IPT; ++j) stage_v[rnk[j]] = val[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = j * BLOCK + tid;
            if (full || i < valid) store_t<NT, V>(gptr<V, SMALL>(job.dst_v, sp[j]), stage_v[i]);
        }
    } else if (STAGE && full) {
        K sk[IPT];
        uint32_t sp[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) sk[j] = lds.stage_k[j * BLOCK + tid];
#pragma unroll
        for (int j = 0; j < IPT; ++j)
            sp[j] = min(lds.gbase[key_digit(sk[j], shift, width)] + j * BLOCK + tid, last);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            store_t<NT, K>(gptr<K, SMALL>(job.dst_k, sp[j]), sk[j]);
            if constexpr (VALS) store_t<NT, V>(gptr<V, SMALL>(job.dst_v, sp[j]), lds.stage_v[j * BLOCK + tid]);
        }
        if constexpr (FUSED) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) atomicAdd(&lds.fused[key_digit(sk[j], job.next_shift, job.next_width)], 1u);
        }
    } else if constexpr (STAGE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = j * BLOCK + tid;
            const K k = lds.stage_k[i];
            const uint32_t p = min(lds.gbase[key_digit(k, shift, width)] + i, last);
            if (i < valid) {
                store_t<NT, K>(gptr<K, SMALL>(job.dst_k, p), k);
                if constexpr (VALS) store_t<NT, V>(gptr<V, SMALL>(job.dst_v, p), lds.stage_v[i]);
                if constexpr (FUSED) atomicAdd(&lds.fused[key_digit(k, job.next_shift, job.next_width)], 1u);
            }
        }
    } else {  // each item from its registers: output slot = digit start + tile rank
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (!full && wslot0 + j * 64 >= valid) continue;
            const uint32_t d = key_digit(key[j], shift, width);
            const uint32_t p = min(lds.gbase[d] + wh[d] + rnk[j], last);
            store_t<NT, K>(gptr<K, SMALL>(job.dst_k, p), key[j]);
            if constexpr (VALS) store_t<NT, V>(gptr<V, SMALL>(job.dst_v, p), val[j]);
        }
    }
    if constexpr (FUSED) {  // the tile's next-digit counts into one copy of the next pass's row
        __syncthreads();
        uint32_t *row = job.next_hist + (blockIdx.x % kFusedCopies) * kFusedBins;
        for (uint32_t d = tid; d < static_cast<uint32_t>(kFusedBins); d += BLOCK) {
            const uint32_t c = lds.fused[d];
            if (c) atomicAdd(&row[d], c);
        }
    }
}

// One block per tile of BLOCK * IPT consecutive items of a single-array
// pass (keys K, values V).  The pass's input is split into chunks (see
// PassPlan); a block claims the next tile of the chunk of the XCD it runs
// on, or of the next chunk with tiles left once that one is exhausted.
// Tiles of a chunk are claimed in order from the chunk's counter, so a
// block only ever waits on tiles claimed before it, by blocks that are
// already running, whichever XCD they run on.  The tiles of a chunk are the
// global grid of TILE-item tiles cut at the chunk's ends, so only a chunk's
// first and last tile can be partial.  The grid needs ctile[nchunks]
// blocks; surplus blocks find every chunk exhausted and exit.  The plan's
// pointers are reinterpreted as K keys and V values.
template <int BITS, int BLOCK, int IPT, typename K, typename V, bool VALS, bool NT, typename S, bool STAGE,
          bool FUSED = false, bool SEQ = false>
__device__ __forceinline__ void onesweep_pass(OnesweepLds<BITS, BLOCK, IPT, K, V, VALS, FUSED, SEQ> &lds,
                                              const SortPlan *__restrict__ plan, int pass, uint32_t n,
                                              S *__restrict__ status, uint32_t *__restrict__ chunk_counter,
                                              uint32_t *__restrict__ error_flag, uint32_t *__restrict__ hist = nullptr) {
    constexpr int TILE = BLOCK * IPT;
    constexpr uint32_t RADIX = 1u << BITS;
    // byte offsets fit in 32 bits (the 32-bit status words serve n < 2^30)
    constexpr bool SMALL = sizeof(S) == 4 && sizeof(K) == 4 && sizeof(V) == 4;
    const PassPlan *pp = plan->pass + pass;
    if (!pp->active) return;
    // this wave's digit counters start at zero (and the fused counts)
    for (uint32_t i = threadIdx.x & 63u; i < RADIX; i += 64) lds.whist[(threadIdx.x >> 6) * RADIX + i] = 0u;
    if constexpr (FUSED)
        for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(kFusedBins); i += BLOCK) lds.fused[i] = 0u;
    if (threadIdx.x == 0)
        claim_tile<TILE>(pp, chunk_counter, lds.claim[0], lds.claim[1], lds.claim[2], lds.claim[3], lds.claim[4]);
    __syncthreads();
    if (lds.claim[0] == kNoTile) return;
    TileJob<K, V> job;
    job.src_k = reinterpret_cast<const K *>(pp->src_k);
    job.src_v = reinterpret_cast<const V *>(pp->src_v);
    job.dst_k = reinterpret_cast<K *>(pp->dst_k);
    job.dst_v = reinterpret_cast<V *>(pp->dst_v);
    job.base = pp->cbase + lds.claim[2] * kChunkRadix;
    job.item0 = lds.claim[3];
    job.shift = pp->shift;
    job.width = pp->width;
    job.tile = lds.claim[0];
    job.first = lds.claim[1];
    job.valid = lds.claim[4];
    job.bound = n;
    job.next_hist = FUSED ? hist + (pass + 1) * kMaxRadix : nullptr;
    job.next_shift = FUSED ? plan->pass[pass + 1].shift : 0u;
    job.next_width = FUSED ? plan->pass[pass + 1].width : 0u;
    onesweep_tile<BITS, BLOCK, IPT, K, V, VALS, NT, S, STAGE, SMALL, FUSED, SEQ>(job, lds, status, error_flag);
}

// The pass over 32-bit keys (with 32-bit values when VALS).  FUSED: the
// pass also counts the next pass's digit of the items it writes into hist's
// row pass + 1 (kFusedCopies copies; see k_plan_fused).
template <int BITS, int BLOCK, int IPT, bool VALS, bool NT, typename S, bool STAGE = true, bool FUSED = false>
__global__ __launch_bounds__(BLOCK) void k_onesweep(const SortPlan *__restrict__ plan, int pass, uint32_t n,
                                                    S *__restrict__ status, uint32_t *__restrict__ chunk_counter,
                                                    uint32_t *__restrict__ error_flag, uint32_t *__restrict__ hist) {
    // 512 x 32 tiles stage keys, then values, through one 64 KiB stage, so
    // that two blocks share a CU (their plain staged pass only)
    constexpr bool SEQ = VALS && BLOCK == 512 && IPT == 32;
    static_assert(!SEQ || (STAGE && !NT && !FUSED), "512 x 32 tiles: the staged pass with plain stores only");
    __shared__ OnesweepLds<BITS, BLOCK, IPT, uint32_t, uint32_t, VALS, FUSED, SEQ> lds;
    onesweep_pass<BITS, BLOCK, IPT, uint32_t, uint32_t, VALS, NT, S, STAGE, FUSED, SEQ>(lds, plan, pass, n, status,
                                                                                       chunk_counter, error_flag, hist);
}

// ---------------------------------------------------------------------------
// copies
// ---------------------------------------------------------------------------

// Moves the result of a sort with exactly one executed pass from the
// temporary back into the caller's arrays.
static __global__ __launch_bounds__(256) void k_copy_back(const SortPlan *__restrict__ plan,
                                                   const uint32_t *__restrict__ tk,
                                                   const uint32_t *__restrict__ tv,
                                                   uint32_t *__restrict__ uk, uint32_t *__restrict__ uv,
                                                   uint32_t n) {
    if (!plan->copy_back) return;
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        uk[i] = tk[i];
        if (uv) uv[i] = tv[i];
    }
}

// Plain streaming copy of 16-byte words, the bandwidth reference: one word
// per thread and one short-lived block per 4 KiB, the form that measured
// fastest on gfx950 (grid-stride loops over fewer blocks were slower).
static __global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                size_t words) {
    const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < words) dst[i] = src[i];
}

// Bandwidth probes, the ceilings the passes are set against (measurement
// only).  Each moves whole 16-byte words: copy with 4 words in flight per
// thread and non-temporal loads and stores over a grid-stride loop; read
// only (an XOR of every word, stored only if it hits a fixed value, so the
// loads cannot be dropped); write only.
constexpr int kProbeWords = 4;  // 16-byte words in flight per thread

static __global__ __launch_bounds__(256) void k_copy16_nt(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          size_t words) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    const v4u *s = reinterpret_cast<const v4u *>(src);
    v4u *d = reinterpret_cast<v4u *>(dst);
    const size_t stride = static_cast<size_t>(gridDim.x) * 256 * kProbeWords;
    for (size_t b = static_cast<size_t>(blockIdx.x) * 256 * kProbeWords; b < words; b += stride) {
        v4u v[kProbeWords];
#pragma unroll
        for (int u = 0; u < kProbeWords; ++u) {
            const size_t i = b + u * 256 + threadIdx.x;
            if (i < words) v[u] = __builtin_nontemporal_load(s + i);
        }
#pragma unroll
        for (int u = 0; u < kProbeWords; ++u) {
            const size_t i = b + u * 256 + threadIdx.x;
            if (i < words) __builtin_nontemporal_store(v[u], d + i);
        }
    }
}

static __global__ __launch_bounds__(256) void k_read16(const uint4 *__restrict__ src, uint32_t *__restrict__ sink,
                                                       size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256 * kProbeWords;
    uint32_t acc = 0;
    for (size_t b = static_cast<size_t>(blockIdx.x) * 256 * kProbeWords; b < words; b += stride) {
        uint4 v[kProbeWords];
#pragma unroll
        for (int u = 0; u < kProbeWords; ++u) {
            const size_t i = b + u * 256 + threadIdx.x;
            v[u] = i < words ? src[i] : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < kProbeWords; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;
}

static __global__ __launch_bounds__(256) void k_write16(uint4 *__restrict__ dst, size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256 * kProbeWords;
    for (size_t b = static_cast<size_t>(blockIdx.x) * 256 * kProbeWords; b < words; b += stride) {
#pragma unroll
        for (int u = 0; u < kProbeWords; ++u) {
            const size_t i = b + u * 256 + threadIdx.x;
            if (i < words) dst[i] = make_uint4(static_cast<uint32_t>(i), 1u, 2u, 3u);
        }
    }
}

static __global__ __launch_bounds__(256) void k_copy4(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                               size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < words; i += stride)
        dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// counter-based input generator (SplitMix64)
// ---------------------------------------------------------------------------

struct GenArgs {
    uint32_t dist;
    uint32_t value_base;
    uint64_t state;
    uint32_t dictionary[16];
    uint64_t thresholds[16];
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t splitmix_word(uint64_t state, uint64_t i) {
    return mix64(state + (i + 1ull) * 0x9E3779B97F4A7C15ull);
}

// Key i of a generated stream (the definition rt_generate documents).
__device__ __forceinline__ uint32_t generate_key(const GenArgs &g, size_t i) {
    if (g.dist == RT_DIST_UNIFORM) return static_cast<uint32_t>(splitmix_word(g.state, i));
    if (g.dist == RT_DIST_AND4) {
        const uint64_t a = splitmix_word(g.state, 2 * i);
        const uint64_t b = splitmix_word(g.state, 2 * i + 1);
        return static_cast<uint32_t>(a) & static_cast<uint32_t>(a >> 32) & static_cast<uint32_t>(b) &
               static_cast<uint32_t>(b >> 32);
    }
    const uint64_t u = splitmix_word(g.state, i) >> 32;
    uint32_t r = 0;
    while (r < 15 && u >= g.thresholds[r]) ++r;
    return g.dictionary[r];
}

static __global__ __launch_bounds__(256) void k_generate(uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                  uint32_t n, GenArgs g) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        keys[i] = generate_key(g, i);
        if (vals) vals[i] = g.value_base + static_cast<uint32_t>(i);
    }
}

}  // namespace rt
