// rt_kernels.h -- gfx950 kernels of the stable LSD radix sort.
//
// One sort is: an upfront read of the keys that builds the digit histograms
// of every pass at once; a planning kernel that turns them into each digit's
// first output slot (exclusive prefix sum), marks passes whose digit is
// constant as skipped and picks source/destination buffers on the device;
// then one "onesweep" kernel per pass.  Each onesweep tile ranks its items
// stably with wave64 ballots, learns the global offset of each digit from
// the tiles before it by decoupled lookback, gathers its items by digit in
// LDS and writes every digit run to HBM as a contiguous burst.
//
// The counting-sort pass is the naive algorithm of Section 3 of Wassenberg &
// Sanders (histogram, exclusive prefix sum, scatter with increment); the pass
// order and stability requirement are Section 4's LSD radix sort.  The LDS
// staging plays the part of Section 2's software write-combining buffers:
// output leaves the chip in runs of consecutive addresses instead of one
// scattered word per item.
#include "rt_internal.h"

namespace rt {

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t popc_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

// Lanes of the wave holding the same BITS-bit digit as this lane: one ballot
// per digit bit, keeping the lanes that agree with this lane on that bit.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
    uint64_t peers = __builtin_amdgcn_read_exec();
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t bit = (d >> b) & 1u;
        const uint64_t set = __builtin_amdgcn_ballot_w64(bit != 0);
        const uint64_t flip = 0ull - static_cast<uint64_t>(bit ^ 1u);  // all ones when bit == 0
        peers &= set ^ flip;
    }
    return peers;
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

// ---------------------------------------------------------------------------
// lookback status words
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

template <typename S>
__device__ __forceinline__ S status_load(const S *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S>
__device__ __forceinline__ void status_store(S *p, S v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool NT>
__device__ __forceinline__ void store_u32(uint32_t *p, uint32_t v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *__restrict__ p, size_t words) {
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

__device__ __forceinline__ void hist_add(uint32_t *s_h, const HistArgs &ha, uint32_t k) {
#pragma unroll
    for (int p = 0; p < kMaxPasses; ++p)
        if (p < static_cast<int>(ha.num_passes))
            atomicAdd(&s_h[ha.lds_offset[p] + ((k >> ha.shift[p]) & ha.mask[p])], 1u);
}

// Counts per pass and digit into hist[p * kMaxRadix + d] (which must start at
// zero); also clears `zero_words` 16-byte words at zero_ptr (the lookback
// state of the passes that follow).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_histogram(const uint32_t *__restrict__ keys, uint32_t n,
                                                     HistArgs ha, uint32_t *__restrict__ hist,
                                                     uint4 *__restrict__ zero_ptr, size_t zero_words) {
    extern __shared__ uint32_t s_h[];
    const uint32_t tid = threadIdx.x;
    for (uint32_t i = tid; i < ha.total_bins; i += BLOCK) s_h[i] = 0u;

    const size_t gthreads = static_cast<size_t>(gridDim.x) * BLOCK;
    const size_t gid = static_cast<size_t>(blockIdx.x) * BLOCK + tid;
    for (size_t i = gid; i < zero_words; i += gthreads) zero_ptr[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();

    // split into an unaligned head, a 16-byte-aligned body and a tail
    const uint32_t mis = static_cast<uint32_t>((reinterpret_cast<uintptr_t>(keys) >> 2) & 3u);
    const uint32_t head = mis ? min(4u - mis, n) : 0u;
    const uint32_t nvec = (n - head) >> 2;
    const uint32_t tail_start = head + (nvec << 2);
    if (blockIdx.x == 0 && tid < head) hist_add(s_h, ha, keys[tid]);
    if (blockIdx.x == 0 && tail_start + tid < n) hist_add(s_h, ha, keys[tail_start + tid]);
    const uint4 *body = reinterpret_cast<const uint4 *>(keys + head);
    for (size_t i = gid; i < nvec; i += gthreads) {
        const uint4 q = body[i];
        hist_add(s_h, ha, q.x);
        hist_add(s_h, ha, q.y);
        hist_add(s_h, ha, q.z);
        hist_add(s_h, ha, q.w);
    }
    __syncthreads();
    for (uint32_t p = 0; p < ha.num_passes; ++p) {
        const uint32_t bins = ha.mask[p] + 1u;
        for (uint32_t d = tid; d < bins; d += BLOCK) {
            const uint32_t c = s_h[ha.lds_offset[p] + d];
            if (c) atomicAdd(&hist[p * kMaxRadix + d], c);
        }
    }
}

// ---------------------------------------------------------------------------
// planning: exclusive prefix sums, pass skipping, buffer assignment
// ---------------------------------------------------------------------------

// One block of 256 threads; thread t covers bins [8t, 8t + 8) of a pass.
__global__ __launch_bounds__(256) void k_plan(PlanArgs a, const uint32_t *__restrict__ hist,
                                              uint32_t *__restrict__ base, SortPlan *__restrict__ plan,
                                              uint32_t *__restrict__ tile_counters, uint32_t direct) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_constant[kMaxPasses];
    const uint32_t tid = threadIdx.x;
    if (tid < kMaxPasses) s_constant[tid] = 0u;
    if (tid <= kMaxPasses) tile_counters[tid] = 0u;  // counters and the error word
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
        for (int i = 0; i < 8; ++i) {
            const uint32_t d = tid * 8 + i;
            if (d < bins) base[p * kMaxRadix + d] = run;
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

// One tile = BLOCK * IPT consecutive items.  Wave w of the tile owns items
// [w * 64 * IPT, (w + 1) * 64 * IPT) of it; lane l holds item j * 64 + l of
// that range in slot j, so slot-by-slot, lane-by-lane processing follows
// input order, which is what makes the ranking stable.
template <int BITS, int BLOCK, int IPT, bool VALS, bool NT, typename S>
__global__ __launch_bounds__(BLOCK) void k_onesweep(const SortPlan *__restrict__ plan, int pass,
                                                    uint32_t n, const uint32_t *__restrict__ pass_base,
                                                    S *__restrict__ status,
                                                    uint32_t *__restrict__ tile_counter,
                                                    uint32_t *__restrict__ error_flag) {
    constexpr int RADIX = 1 << BITS;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * IPT;
    constexpr int WAVE_ITEMS = 64 * IPT;
    constexpr int R = RADIX >= BLOCK ? RADIX / BLOCK : 1;  // digits per owning thread
    constexpr int DT = RADIX / R;                            // owning threads
    using St = Status<S>;

    const PassPlan pp = plan->pass[pass];
    if (!pp.active) return;

    __shared__ uint32_t s_stage[TILE];
    __shared__ uint32_t s_whist[WAVES * RADIX];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_wsum[WAVES];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    if (tid == 0) s_tile = atomicAdd(tile_counter + pass, 1u);
    for (uint32_t i = tid; i < WAVES * RADIX; i += BLOCK) s_whist[i] = 0u;
    __syncthreads();

    const uint32_t tile = s_tile;
    const uint32_t shift = pp.shift;
    const uint32_t mask = (1u << pp.width) - 1u;
    const size_t tile_base = static_cast<size_t>(tile) * TILE;
    if (tile_base >= n) return;  // only if the tile counter was not cleared
    const uint32_t valid = static_cast<uint32_t>(min(static_cast<size_t>(TILE), n - tile_base));
    const bool full = valid == static_cast<uint32_t>(TILE);
    const uint32_t wslot0 = wave * WAVE_ITEMS + lane;  // tile index of this lane's slot 0

    // ---- load (coalesced: each slot of a wave is 256 consecutive bytes)
    uint32_t key[IPT];
    uint32_t val[VALS ? IPT : 1];
    {
        const uint32_t *sk = pp.src_k + tile_base + wslot0;
        const uint32_t *sv = VALS ? pp.src_v + tile_base + wslot0 : nullptr;
        if (full) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) key[j] = sk[j * 64];
            if constexpr (VALS) {
#pragma unroll
                for (int j = 0; j < IPT; ++j) val[j] = sv[j * 64];
            }
        } else {
#pragma unroll
            for (int j = 0; j < IPT; ++j) key[j] = (wslot0 + j * 64 < valid) ? sk[j * 64] : 0u;
            if constexpr (VALS) {
#pragma unroll
                for (int j = 0; j < IPT; ++j) val[j] = (wslot0 + j * 64 < valid) ? sv[j * 64] : 0u;
            }
        }
    }

    // ---- stable rank inside the wave, per-wave digit counts in LDS
    // Items past the end of the array take the last digit, so they rank
    // behind every real item of the tile and are never written.
    uint32_t rnk[IPT];
    uint32_t *wh = s_whist + wave * RADIX;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = (key[j] >> shift) & mask;
        if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
        const uint64_t peers = match_digit<BITS>(d);
        const uint32_t below = popc_below(peers);
        const uint32_t cnt = wh[d];
        rnk[j] = cnt + below;
        if (below == 0) wh[d] = cnt + static_cast<uint32_t>(__popcll(peers));
        compiler_fence();
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
    {
        uint32_t run = texcl;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            dexcl[r] = run;
            run += tid < DT ? tcount[r] : 0u;
        }
    }
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int w = 0; w < WAVES; ++w) s_whist[w * RADIX + tid * R + r] += dexcl[r];
    }
    __syncthreads();

    // ---- gather keys by digit in LDS (tile rank = digit start + earlier
    // waves + rank inside the wave)
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = (key[j] >> shift) & mask;
        if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
        const uint32_t r = wh[d] + rnk[j];
        rnk[j] = r;
        s_stage[r] = key[j];
    }

    // ---- decoupled lookback: sum the counts of earlier tiles per digit
    if (tid < DT) {
        uint32_t excl[R];
        int32_t at[R];
        bool done[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            excl[r] = 0;
            at[r] = static_cast<int32_t>(tile) - 1;
            done[r] = tile == 0;
        }
        bool all_done = tile == 0;
        uint32_t idle = 0;
        while (!all_done) {
            all_done = true;
            bool progressed = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (done[r]) continue;
                const S s = status_load(status + static_cast<size_t>(at[r]) * RADIX + tid * R + r);
                const uint32_t f = St::flag(s);
                if (f != 0u) {
                    progressed = true;
                    excl[r] += St::count(s);
                    if (f == kFlagIncl)
                        done[r] = true;
                    else
                        --at[r];
                }
                all_done = all_done && done[r];
            }
            if (!all_done && !progressed) {
                __builtin_amdgcn_s_sleep(1);
                // Every earlier tile publishes within microseconds; a wait
                // this long means broken state, so flag it and stop waiting
                // rather than hold the GPU.
                if (++idle > kLookbackSpinLimit) {
                    atomicOr(error_flag, kErrLookbackTimeout);
                    break;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            if (tile != 0)
                status_store(status + static_cast<size_t>(tile) * RADIX + d,
                             St::make(kFlagIncl, excl[r] + tcount[r]));
            s_gbase[d] = pass_base[d] + excl[r] - dexcl[r];
        }
    }
    __syncthreads();

    // ---- scatter keys: consecutive LDS slots of one digit go to consecutive
    // output addresses
    uint32_t pos[VALS ? IPT : 1];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t i = j * BLOCK + tid;
        const uint32_t k = s_stage[i];
        const uint32_t p = s_gbase[(k >> shift) & mask] + i;
        if (VALS) pos[VALS ? j : 0] = p;
        // p < n holds for every real item; the test keeps a logic error from
        // ever becoming a stray store
        if ((full || i < valid) && p < n) store_u32<NT>(pp.dst_k + p, k);
    }
    if constexpr (VALS) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) s_stage[rnk[j]] = val[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t i = j * BLOCK + tid;
            if ((full || i < valid) && pos[j] < n) store_u32<NT>(pp.dst_v + pos[j], s_stage[i]);
        }
    }
}

// ---------------------------------------------------------------------------
// copies
// ---------------------------------------------------------------------------

// Moves the result of a sort with exactly one executed pass from the
// temporary back into the caller's arrays.
__global__ __launch_bounds__(256) void k_copy_back(const SortPlan *__restrict__ plan,
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

// Plain streaming copy of 16-byte words, the bandwidth reference.
__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                size_t words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < words; i += stride)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_copy4(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
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

__global__ __launch_bounds__(256) void k_generate(uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                  uint32_t n, GenArgs g) {
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        uint32_t k;
        if (g.dist == RT_DIST_UNIFORM) {
            k = static_cast<uint32_t>(splitmix_word(g.state, i));
        } else if (g.dist == RT_DIST_AND4) {
            const uint64_t a = splitmix_word(g.state, 2 * i);
            const uint64_t b = splitmix_word(g.state, 2 * i + 1);
            k = static_cast<uint32_t>(a) & static_cast<uint32_t>(a >> 32) & static_cast<uint32_t>(b) &
                static_cast<uint32_t>(b >> 32);
        } else {
            const uint64_t u = splitmix_word(g.state, i) >> 32;
            uint32_t r = 0;
            while (r < 15 && u >= g.thresholds[r]) ++r;
            k = g.dictionary[r];
        }
        keys[i] = k;
        if (vals) vals[i] = g.value_base + static_cast<uint32_t>(i);
    }
}

}  // namespace rt
