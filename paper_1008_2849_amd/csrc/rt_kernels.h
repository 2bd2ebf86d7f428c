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

// Exclusive prefix sum of v over the block; every thread must call it.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t *s_wsum) {
    constexpr int WAVES = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w)
        if (w < wave) before += s_wsum[w];
    return before + x - v;
}

template <bool NT>
__device__ __forceinline__ void store_g(g_u32 *p, uint32_t v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
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

// ---------------------------------------------------------------------------
// upfront histograms of all passes (one read of the keys)
// ---------------------------------------------------------------------------

struct HistArgs {
    uint32_t num_passes;
    uint32_t shift[kMaxPasses];
    uint32_t mask[kMaxPasses];
    uint32_t lds_offset[kMaxPasses];
    uint32_t total_bins;
};

// Counts per pass and digit into hist[p * kMaxRadix + d], which must start at
// zero.  A block keeps C copies of the counters of all passes in LDS, one
// per lane class (lane mod C), in rows of total_bins + 1 words: lanes that
// hit the same digit then add into C different words in C different banks,
// so skewed keys no longer serialise on one LDS address.  Before counting a
// wave's batch of 64 * U keys, one test per pass checks whether the whole
// batch shares that pass's digit (constant bytes, runs of equal keys); such
// a digit is counted with a single add.  Keys are read in 256-byte slots.
template <int BLOCK, int C>
__global__ __launch_bounds__(BLOCK) void k_histogram(const uint32_t *__restrict__ keys, uint32_t n,
                                                     HistArgs ha, uint32_t *__restrict__ hist) {
    constexpr int WAVES = BLOCK / 64;
    constexpr int U = 16;  // slots in flight per lane (8 measured 18 % slower on 2^28 keys)
    extern __shared__ uint32_t s_h[];  // C rows of total_bins + 1 counters
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
                if (__builtin_amdgcn_ballot_w64(((differ >> ha.shift[p]) & ha.mask[p]) != 0u) == 0u) {
                    if (lane == 0) atomicAdd(&hp[(k0 >> ha.shift[p]) & ha.mask[p]], static_cast<uint32_t>(64 * U));
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) atomicAdd(&hp[(k[u] >> ha.shift[p]) & ha.mask[p]], 1u);
                }
            }
        } else {  // the ragged end of the array
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = base + u * 64 + lane;
                if (i >= n) continue;
                const uint32_t key = keys[i];
                for (int p = 0; p < static_cast<int>(ha.num_passes); ++p)
                    atomicAdd(&h[ha.lds_offset[p] + ((key >> ha.shift[p]) & ha.mask[p])], 1u);
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
        atomicAdd(&hist[p * kMaxRadix + (i - ha.lds_offset[p])], c);
    }
}

// ---------------------------------------------------------------------------
// planning: exclusive prefix sums, pass skipping, buffer assignment
// ---------------------------------------------------------------------------

// One block of 256 threads; thread t covers bins [8t, 8t + 8) of a pass.
// Also clears the tile counters of the passes and the error word after them.
static __global__ __launch_bounds__(256) void k_plan(PlanArgs a, const uint32_t *__restrict__ hist,
                                              uint32_t *__restrict__ base, SortPlan *__restrict__ plan,
                                              uint32_t *__restrict__ tile_counters, uint32_t direct) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_constant[kMaxPasses];
    const uint32_t tid = threadIdx.x;
    if (tid < kMaxPasses) {
        s_constant[tid] = 0u;
        tile_counters[tid] = 0u;
    }
    if (tid == kMaxPasses) tile_counters[kMaxPasses] = 0u;  // the error word
    __syncthreads();
    for (uint32_t p = 0; p < a.num_passes; ++p) {
        const uint32_t bins = 1u << a.width[p];
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
        pp.pad = 0;
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
    }
    plan->executed = executed;
    plan->copy_back = (!direct && executed == 1) ? 1u : 0u;
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

template <typename S>
__device__ __forceinline__ uint32_t lookback_digit(const S *__restrict__ status, int32_t tile, uint32_t digit,
                                                   int radix, uint32_t *__restrict__ error_flag) {
    using St = Status<S>;
    uint32_t excl = 0;
    int32_t at = tile - 1;  // the nearest tile not yet accounted for
    uint32_t idle = 0, nap = 1;
    while (at >= 0) {
        S w[kLookbackBatch];
#pragma unroll
        for (int b = 0; b < kLookbackBatch; ++b)
            w[b] = (at - b >= 0) ? status_load(status + static_cast<size_t>(at - b) * radix + digit) : S(0);
        bool finished = false, stalled = false;
        int32_t consumed = 0;
#pragma unroll
        for (int b = 0; b < kLookbackBatch; ++b) {
            if (finished || stalled || at - b < 0) continue;
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

// One block per tile of BLOCK * IPT consecutive items, claimed in order from
// an atomic counter (so a block only ever waits on tiles claimed before it,
// by blocks that are already running).  Wave w of the tile owns items
// [w * 64 * IPT, (w + 1) * 64 * IPT) of it and lane l holds item j * 64 + l
// of that range in slot j, so slot-by-slot, lane-by-lane processing follows
// input order, which makes the ranking stable.
//
// Phases: load keys and values -> rank every item inside its wave (ballot
// match + per-wave digit counters in LDS) -> per-digit tile counts,
// published as this tile's aggregate -> tile-local digit offsets -> gather
// keys and values by digit in LDS -> lookback for the global offset of each
// digit -> write every digit run to consecutive output addresses.
//
// STAGE = false drops the gather: every item is written straight from its
// registers to its output slot, so a wave's stores scatter over the digit
// runs.  This is the pass without write-combining (the paper's "VM only"
// counterpart), kept to measure what the staging buys.
template <int BITS, int BLOCK, int IPT, bool VALS, bool NT, typename S, bool STAGE = true>
__global__ __launch_bounds__(BLOCK) void k_onesweep(const SortPlan *__restrict__ plan, int pass, uint32_t n,
                                                    const uint32_t *__restrict__ pass_base, S *__restrict__ status,
                                                    uint32_t *__restrict__ tile_counter,
                                                    uint32_t *__restrict__ error_flag) {
    constexpr int RADIX = 1 << BITS;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * IPT;
    constexpr int WAVE_ITEMS = 64 * IPT;
    constexpr int R = RADIX >= BLOCK ? RADIX / BLOCK : 1;  // digits per owning thread
    constexpr int DT = RADIX / R;                            // owning threads
    constexpr bool SMALL = sizeof(S) == 4;                    // n < 2^30
    using St = Status<S>;

    const PassPlan pp = plan->pass[pass];
    if (!pp.active) return;

    __shared__ uint32_t s_stage_k[TILE];
    __shared__ uint32_t s_stage_v[VALS ? TILE : 1];
    // per-wave digit counters, then a 64-word scratch row per wave that
    // absorbs the counter writes of non-leader lanes
    __shared__ uint32_t s_whist[WAVES * RADIX + WAVES * 64];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_wsum[WAVES];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t shift = pp.shift;
    const uint32_t width = pp.width;
    const uint32_t wslot0 = wave * WAVE_ITEMS + lane;  // tile index of this lane's slot 0
    uint32_t *wh = s_whist + wave * RADIX;
    uint32_t *scratch = s_whist + WAVES * RADIX + wave * 64 + lane;

    for (uint32_t i = lane; i < RADIX; i += 64) wh[i] = 0u;  // this wave's counters
    if (tid == 0) s_tile = atomicAdd(tile_counter + pass, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const size_t tile_base = static_cast<size_t>(tile) * TILE;
    if (tile_base >= n) return;  // only if the tile counter was not cleared
    const uint32_t valid = static_cast<uint32_t>(min(static_cast<size_t>(TILE), n - tile_base));
    const bool full = valid == static_cast<uint32_t>(TILE);

    // ---- load (each slot of a wave is 256 consecutive bytes).  In a full
    // tile the values are loaded halfway through the ranking below, which
    // needs only the keys: the tile's key loads then do not queue behind its
    // value loads (2 % faster passes than loading both here).
    uint32_t key[IPT];
    uint32_t val[VALS ? IPT : 1];
    if (full) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) key[j] = *gelem<SMALL>(pp.src_k, tile_base + wslot0 + j * 64);
    } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j)
            key[j] = (wslot0 + j * 64 < valid) ? *gelem<SMALL>(pp.src_k, tile_base + wslot0 + j * 64) : 0u;
        if constexpr (VALS) {
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                val[j] = (wslot0 + j * 64 < valid) ? *gelem<SMALL>(pp.src_v, tile_base + wslot0 + j * 64) : 0u;
        }
    }

    // ---- stable rank inside the wave, per-wave digit counts in LDS.
    // Items past the end take the last digit, so they rank behind every real
    // item of the tile and are never written.
    uint32_t rnk[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = __builtin_amdgcn_ubfe(key[j], shift, width);
        if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
        uint32_t lo, hi;
        match_digit<BITS>(d, lo, hi);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
        const uint32_t cnt = wh[d];
        rnk[j] = cnt + below;
        // the first lane of each digit advances the counter; the others
        // write their private scratch word instead
        uint32_t *dst = below == 0 ? wh + d : scratch;
        *dst = cnt + __builtin_popcount(lo) + __builtin_popcount(hi);
        compiler_fence();
        if constexpr (VALS) {
            if (full && j == IPT / 2 - 1) {
#pragma unroll
                for (int q = 0; q < IPT; ++q) val[q] = *gelem<SMALL>(pp.src_v, tile_base + wslot0 + q * 64);
            }
        }
    }
    __syncthreads();

    // ---- per digit: counts of earlier waves, tile count, publish aggregate
    uint32_t tcount[R];
    uint32_t tsum = 0;
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            uint32_t run = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint32_t c = s_whist[w * RADIX + d];
                s_whist[w * RADIX + d] = run;
                run += c;
            }
            tcount[r] = run;
            tsum += run;
            status_store(status + static_cast<size_t>(tile) * RADIX + d,
                         St::make(tile == 0 ? kFlagIncl : kFlagAgg, run));
        }
    }
    const uint32_t texcl = block_exclusive_sum<BLOCK>(tid < DT ? tsum : 0u, s_wsum);
    uint32_t dexcl[R];
    if (tid < DT) {
        uint32_t run = texcl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            dexcl[r] = run;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) s_whist[w * RADIX + d] += run;
            run += tcount[r];
        }
    }
    __syncthreads();

    // ---- gather keys and values by digit in LDS (tile rank = digit start +
    // earlier waves + rank inside the wave)
    if constexpr (STAGE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            uint32_t d = __builtin_amdgcn_ubfe(key[j], shift, width);
            if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
            const uint32_t r = wh[d] + rnk[j];
            s_stage_k[r] = key[j];
            if constexpr (VALS) s_stage_v[r] = val[j];
        }
    }

    // ---- lookback: the count of each digit in all earlier tiles
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            const uint32_t excl = lookback_digit<S>(status, static_cast<int32_t>(tile), d, RADIX, error_flag);
            if (tile != 0)
                status_store(status + static_cast<size_t>(tile) * RADIX + d, St::make(kFlagIncl, excl + tcount[r]));
            // LDS slot i of digit d goes to output slot s_gbase[d] + i
            s_gbase[d] = pass_base[d] + excl - dexcl[r];
        }
    }
    __syncthreads();

    // ---- scatter: consecutive LDS slots of one digit go to consecutive
    // output addresses.  The clamp to n - 1 costs one op and keeps a logic
    // error from ever turning into a store outside the array.
    if constexpr (STAGE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = j * BLOCK + tid;
            const uint32_t k = s_stage_k[i];
            const uint32_t p = min(s_gbase[__builtin_amdgcn_ubfe(k, shift, width)] + i, n - 1u);
            if (full || i < valid) {
                store_g<NT>(gelem<SMALL>(pp.dst_k, p), k);
                if constexpr (VALS) store_g<NT>(gelem<SMALL>(pp.dst_v, p), s_stage_v[i]);
            }
        }
    } else {  // each item from its registers: output slot = digit start + tile rank
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (!full && wslot0 + j * 64 >= valid) continue;
            const uint32_t d = __builtin_amdgcn_ubfe(key[j], shift, width);
            const uint32_t p = min(s_gbase[d] + wh[d] + rnk[j], n - 1u);
            store_g<NT>(gelem<SMALL>(pp.dst_k, p), key[j]);
            if constexpr (VALS) store_g<NT>(gelem<SMALL>(pp.dst_v, p), val[j]);
        }
    }
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
