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

// The pass over 64-bit keys with values of VW 32-bit words (0, 1 or 2):
// the single-array pass of k_onesweep on wider items.
template <int BITS, int BLOCK, int IPT, int VW, typename S>
__global__ __launch_bounds__(BLOCK) void k_onesweep64(const SortPlan *__restrict__ plan, int pass, uint32_t n,
                                                      S *__restrict__ status, uint32_t *__restrict__ chunk_counter,
                                                      uint32_t *__restrict__ error_flag) {
    typedef typename ValWord<VW>::type V;
    // a tile whose keys and values do not fit the LDS together stages the
    // keys, then the values through the same space
    constexpr bool SEQ = VW > 0 && static_cast<size_t>(BLOCK) * IPT * (sizeof(uint64_t) + sizeof(V)) > 128 * 1024;
    __shared__ OnesweepLds<BITS, BLOCK, IPT, uint64_t, V, (VW > 0), false, SEQ> lds;
    onesweep_pass<BITS, BLOCK, IPT, uint64_t, V, (VW > 0), false, S, true, false, SEQ>(lds, plan, pass, n, status,
                                                                                       chunk_counter, error_flag);
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
