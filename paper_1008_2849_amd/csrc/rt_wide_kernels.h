// rt_wide_kernels.h -- gfx950 kernels of the LSD radix sort of 64-bit keys.
//
// The sort is the one of rt_kernels.h with K = 64-bit keys (Section 4 allows
// larger items than one 64-bit key-value word): an upfront read builds the
// digit histograms of every pass, the shared planning kernel turns them into
// digit offsets, skips constant digits and assigns buffers, and one onesweep
// kernel per executed pass ranks, looks back, stages by digit in LDS and
// writes each digit run as consecutive addresses.  Values ride along as one
// or two 32-bit words per item (VW), or are absent (VW = 0).
//
// What differs from the 32-bit kernels: keys live in registers and LDS as
// 64-bit words (a tile of 8K items stages 64 KiB of keys), a digit is taken
// from the whole 64-bit key (an 11-bit digit may straddle its two halves),
// and global addresses are formed in 64 bits.
#include "rt_kernels.h"

namespace rt {

typedef __attribute__((address_space(1))) uint64_t g_u64;

template <int VW>
struct ValWord {
    typedef uint32_t type;  // VW = 0 (unused) or 1
};
template <>
struct ValWord<2> {
    typedef uint64_t type;  // two 32-bit words moved as one
};

__device__ __forceinline__ uint32_t digit64(uint64_t key, uint32_t shift, uint32_t mask) {
    return static_cast<uint32_t>(key >> shift) & mask;
}

// ---------------------------------------------------------------------------
// upfront histograms of all passes (one read of the 64-bit keys)
// ---------------------------------------------------------------------------

// As k_histogram: C lane-class copies of every pass's counters in padded LDS
// rows, and a wave batch of 64 * U keys that shares a pass's digit counted
// with one add.  hist[p * kMaxRadix + d] must start at zero.  CHUNKED: the
// per-chunk counts of k_histogram's CHUNKED form, for the XCD chunks of the
// 64-bit passes (a wave batch of 512 keys never straddles a chunk of pass 0:
// the bounds are multiples of the 8K tile).
template <int BLOCK, int C, bool CHUNKED>
__device__ __forceinline__ void histogram64_body(const uint64_t *__restrict__ keys, uint32_t n, const HistArgs &ha,
                                                 uint32_t *__restrict__ hist, uint32_t *s_h) {
    constexpr int WAVES = BLOCK / 64;
    constexpr int U = 8;
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
        if (base + wave_span <= n) {
            uint64_t k[U];
#pragma unroll
            for (int u = 0; u < U; ++u) k[u] = keys[base + u * 64 + lane];
            const uint64_t k0 = (static_cast<uint64_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(k[0] >> 32)))
                                 << 32) |
                                __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(k[0]));
            uint64_t differ = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) differ |= k[u] ^ k0;
#pragma unroll
            for (int p = 0; p < kMaxPasses; ++p) {
                if (p >= static_cast<int>(ha.num_passes)) break;
                uint32_t *hp = h + ha.lds_offset[p];
                const uint32_t sh = ha.shift[p], m = ha.mask[p];
                if (!CHUNKED || p == 0) {
                    if constexpr (CHUNKED) hp += pos_chunk(ha, base) * (m + 1u);
                    if (__builtin_amdgcn_ballot_w64(digit64(differ, sh, m) != 0u) == 0u) {
                        if (lane == 0) atomicAdd(&hp[digit64(k0, sh, m)], static_cast<uint32_t>(64 * U));
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[digit64(k[u], sh, m)], 1u);
                    }
                } else {
                    const uint32_t cs = ha.shift[p - 1] + ha.cshift[p - 1];
                    const uint32_t cm = ha.mask[p - 1] >> ha.cshift[p - 1];
                    const uint32_t w = 32u - __builtin_clz(m);
                    if (__builtin_amdgcn_ballot_w64((digit64(differ, sh, m) | digit64(differ, cs, cm)) != 0u) == 0u) {
                        if (lane == 0)
                            atomicAdd(&hp[(digit64(k0, cs, cm) << w) | digit64(k0, sh, m)], static_cast<uint32_t>(64 * U));
                    } else {
#pragma unroll
                        for (int u = 0; u < U; ++u) atomicAdd(&hp[(digit64(k[u], cs, cm) << w) | digit64(k[u], sh, m)], 1u);
                    }
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const size_t i = base + u * 64 + lane;
                if (i >= n) continue;
                const uint64_t key = keys[i];
                for (int p = 0; p < static_cast<int>(ha.num_passes); ++p) {
                    uint32_t bin = digit64(key, ha.shift[p], ha.mask[p]);
                    if constexpr (CHUNKED) {
                        const uint32_t w = 32u - __builtin_clz(ha.mask[p]);
                        const uint32_t x = p == 0 ? pos_chunk(ha, i)
                                                  : digit64(key, ha.shift[p - 1], ha.mask[p - 1]) >> ha.cshift[p - 1];
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

template <int BLOCK, int C>
__global__ __launch_bounds__(BLOCK) void k_histogram64(const uint64_t *__restrict__ keys, uint32_t n, HistArgs ha,
                                                       uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t s_h[];
    histogram64_body<BLOCK, C, false>(keys, n, ha, hist, s_h);
}

template <int BLOCK, int C>
__global__ __launch_bounds__(BLOCK) void k_histogram64_chunked(const uint64_t *__restrict__ keys, uint32_t n,
                                                               HistArgs ha, uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t s_h[];
    histogram64_body<BLOCK, C, true>(keys, n, ha, hist, s_h);
}

// Per-chunk counts (CC copies, args hc) if the probe chose them, else plain
// counts (CP copies, hp): see k_histogram_auto.
template <int BLOCK, int CP, int CC>
__global__ __launch_bounds__(BLOCK) void k_histogram64_auto(const uint64_t *__restrict__ keys, uint32_t n, HistArgs hp,
                                                            HistArgs hc, const uint32_t *__restrict__ mode,
                                                            uint32_t *__restrict__ hist) {
    extern __shared__ uint32_t s_h[];
    if (*mode != 0u)
        histogram64_body<BLOCK, CC, true>(keys, n, hc, hist, s_h);
    else
        histogram64_body<BLOCK, CP, false>(keys, n, hp, hist, s_h);
}

// ---------------------------------------------------------------------------
// onesweep counting-sort pass over 64-bit keys
// ---------------------------------------------------------------------------

// The structure of k_onesweep: tiles claimed in XCD chunks (claim_tile);
// wave w owns items [w * 64 * IPT, (w + 1) * 64 * IPT) of the tile
// and lane l holds item j * 64 + l in slot j, so the ballot ranking follows
// input order (stable); per-digit tile counts are published as the tile's
// aggregate, the tile is staged by digit in LDS, the lookback gives each
// digit's offset among earlier tiles, and consecutive LDS slots of a digit
// go to consecutive output addresses.  The plan's pointers are reinterpreted
// as 64-bit keys and VW-word values.
template <int BITS, int BLOCK, int IPT, int VW, typename S>
__global__ __launch_bounds__(BLOCK) void k_onesweep64(const SortPlan *__restrict__ plan, int pass, uint32_t n,
                                                      S *__restrict__ status, uint32_t *__restrict__ chunk_counter,
                                                      uint32_t *__restrict__ error_flag) {
    constexpr int RADIX = 1 << BITS;
    constexpr int WAVES = BLOCK / 64;
    constexpr int TILE = BLOCK * IPT;
    constexpr int WAVE_ITEMS = 64 * IPT;
    constexpr int R = RADIX >= BLOCK ? RADIX / BLOCK : 1;
    constexpr int DT = RADIX / R;
    constexpr bool VALS = VW > 0;
    typedef typename ValWord<VW>::type V;
    typedef __attribute__((address_space(1))) V g_v;
    using St = Status<S>;

    const PassPlan pp = plan->pass[pass];
    if (!pp.active) return;

    __shared__ uint64_t s_stage_k[TILE];
    __shared__ V s_stage_v[VALS ? TILE : 1];
    __shared__ uint32_t s_whist[WAVES * RADIX + WAVES * 64];
    __shared__ uint32_t s_gbase[RADIX];
    __shared__ uint32_t s_wsum[WAVES];
    __shared__ uint32_t s_tile, s_first, s_chunk, s_lo, s_valid;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const uint32_t wave = tid >> 6;
    const uint32_t shift = pp.shift;
    const uint32_t mask = (1u << pp.width) - 1u;
    const uint32_t wslot0 = wave * WAVE_ITEMS + lane;
    uint32_t *wh = s_whist + wave * RADIX;
    uint32_t *scratch = s_whist + WAVES * RADIX + wave * 64 + lane;
    const g_u64 *src_k = (const g_u64 *)pp.src_k;
    g_u64 *dst_k = (g_u64 *)pp.dst_k;
    const g_v *src_v = (const g_v *)pp.src_v;
    g_v *dst_v = (g_v *)pp.dst_v;

    for (uint32_t i = lane; i < RADIX; i += 64) wh[i] = 0u;
    if (tid == 0) claim_tile<TILE>(plan->pass + pass, chunk_counter, s_tile, s_first, s_chunk, s_lo, s_valid);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile == kNoTile) return;
    const int32_t first = static_cast<int32_t>(s_first);
    const size_t tile_base = s_lo;
    const uint32_t valid = s_valid;
    const bool full = valid == static_cast<uint32_t>(TILE);
    const uint32_t *pass_base = pp.cbase + s_chunk * kChunkRadix;

    uint64_t key[IPT];
    V val[VALS ? IPT : 1];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t i = wslot0 + j * 64;
        key[j] = (full || i < valid) ? src_k[tile_base + i] : 0ull;
    }
    if constexpr (VALS) {  // a full tile loads its values halfway through the ranking
        if (!full) {
#pragma unroll
            for (int j = 0; j < IPT; ++j) {
                const uint32_t i = wslot0 + j * 64;
                val[j] = i < valid ? src_v[tile_base + i] : V(0);
            }
        }
    }

    // stable rank inside the wave; items past the end take the last digit
    uint32_t rnk[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = digit64(key[j], shift, mask);
        if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
        uint32_t lo, hi;
        match_digit<BITS>(d, lo, hi);
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
        const uint32_t cnt = wh[d];
        rnk[j] = cnt + below;
        uint32_t *dst = below == 0 ? wh + d : scratch;
        *dst = cnt + __builtin_popcount(lo) + __builtin_popcount(hi);
        compiler_fence();
        if constexpr (VALS) {
            if (full && j == IPT / 2 - 1) {
#pragma unroll
                for (int q = 0; q < IPT; ++q) val[q] = src_v[tile_base + wslot0 + q * 64];
            }
        }
    }
    __syncthreads();

    // per digit: earlier waves' counts, tile count, publish the aggregate
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
            if (d == RADIX - 1) run -= TILE - valid;  // a partial tile's empty slots are not items
            tcount[r] = run;
            tsum += run;
            status_store(status + static_cast<size_t>(tile) * RADIX + d,
                         St::make(static_cast<int32_t>(tile) == first ? kFlagIncl : kFlagAgg, run));
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

    // gather by digit in LDS
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        uint32_t d = digit64(key[j], shift, mask);
        if (!full && wslot0 + j * 64 >= valid) d = RADIX - 1;
        const uint32_t r = wh[d] + rnk[j];
        s_stage_k[r] = key[j];
        if constexpr (VALS) s_stage_v[r] = val[j];
    }

    // lookback
    if (tid < DT) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t d = tid * R + r;
            const uint32_t excl = lookback_digit<S>(status, static_cast<int32_t>(tile), first, d, RADIX, error_flag);
            if (static_cast<int32_t>(tile) != first)
                status_store(status + static_cast<size_t>(tile) * RADIX + d, St::make(kFlagIncl, excl + tcount[r]));
            s_gbase[d] = pass_base[d] + excl - dexcl[r];
        }
    }
    __syncthreads();

    // scatter; the clamp keeps a logic error from storing outside the array.
    // A full tile needs no per-slot guard, so its LDS reads issue together.
    if (full) {
        uint64_t sk[IPT];
        uint32_t sp[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) sk[j] = s_stage_k[j * BLOCK + tid];
#pragma unroll
        for (int j = 0; j < IPT; ++j) sp[j] = min(s_gbase[digit64(sk[j], shift, mask)] + j * BLOCK + tid, n - 1u);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            dst_k[sp[j]] = sk[j];
            if constexpr (VALS) dst_v[sp[j]] = s_stage_v[j * BLOCK + tid];
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t i = j * BLOCK + tid;
        const uint64_t k = s_stage_k[i];
        const uint32_t p = min(s_gbase[digit64(k, shift, mask)] + i, n - 1u);
        if (i < valid) {
            dst_k[p] = k;
            if constexpr (VALS) dst_v[p] = s_stage_v[i];
        }
    }
}

// Moves the result of a sort with exactly one executed pass from the
// temporary back into the caller's arrays: key_words and val_words 32-bit
// words per item.
static __global__ __launch_bounds__(256) void k_copy_back_words(const SortPlan *__restrict__ plan,
                                                               const uint32_t *__restrict__ tk,
                                                               const uint32_t *__restrict__ tv,
                                                               uint32_t *__restrict__ uk, uint32_t *__restrict__ uv,
                                                               size_t key_words, size_t val_words) {
    if (!plan->copy_back) return;
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < key_words; i += stride) uk[i] = tk[i];
    for (size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; i < val_words; i += stride) uv[i] = tv[i];
}

}  // namespace rt
