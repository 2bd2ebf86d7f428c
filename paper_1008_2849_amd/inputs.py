"""Seeded synthetic inputs for the sort workloads.

This module only draws input data; it holds none of the sort's arithmetic.
Both sides of every parity check (the GPU library and the CPU oracle) are fed
from here, and the benchmark uses it too.

The paper's workload is N uniform 32-bit keys from a seeded generator
(Section 5, performance evaluation); the skewed, batched and serving
workloads add shapes the paper does not measure (low-entropy keys, a
constant top byte, a 16-key Zipf dictionary, many uneven segments, Poisson
arrivals).  Host-side draws use numpy's PCG64 (``default_rng(seed)``); the
paper's WELL512 stream and seed are not given, and only the distribution
matters.

``counter_keys`` is a counter-based form of the same distributions, defined
on SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): word i of a stream with state s is
``mix64(s + (i + 1) * 0x9E3779B97F4A7C15)``.  The GPU library implements the
same published definition in its device generator, so request inputs can be
made on the device and re-made here, bit for bit, for checking.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional, Tuple

import numpy as np

U32 = np.uint32
MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15

# Fixed seeds of the workloads (one per configuration).
SEED_KEYS_1M = 1          # 2^20 uniform keys, keys only
SEED_PAIRS_256M = 2       # 2^28 uniform key/value pairs
SEED_AND = {2: 31, 4: 32, 8: 33}   # AND of k uniform words, 2^26 pairs
SEED_TOP_BYTE = 34        # 24 significant bits, 2^26 pairs
SEED_ZIPF16 = 35          # 16 distinct keys, Zipf s = 1.2, 2^26 pairs
SEED_BATCHED = 4          # 4096 segments
SEED_SERVING = 5          # serving request stream
SEED_PAIRS64_256M = 6     # 2^28 uniform 64-bit keys with 32-bit index values
SEED_TABLE1 = 7           # 2^26 (64 Mi) uniform keys: the paper's own N, keys only and pairs
SEED_KEYS_256M = 8        # 2^28 uniform keys, keys only

# Distribution ids shared with the device generator.
DIST_UNIFORM = 0
DIST_AND4 = 1
DIST_ZIPF16 = 2
DIST_NAMES = {DIST_UNIFORM: "uniform", DIST_AND4: "and4", DIST_ZIPF16: "zipf16"}


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def uniform_keys(n: int, seed: int) -> np.ndarray:
    """n keys uniform over [0, 2^32)."""
    return _rng(seed).integers(0, 2**32, size=n, dtype=U32)


def uniform_keys64(n: int, seed: int) -> np.ndarray:
    """n keys uniform over [0, 2^64)."""
    return _rng(seed).integers(0, 1 << 64, size=n, dtype=np.uint64)


def keys64(kind: str, n: int, seed: int) -> np.ndarray:
    """64-bit keys: uniform; `small` (below 2^20, so the high digits are
    constant); `high` (only the top 16 bits vary); `low32` (the high half is
    zero); `and2` (AND of two uniform words)."""
    u = uniform_keys64(n, seed)
    if kind == "uniform":
        return u
    if kind == "small":
        return u >> np.uint64(44)
    if kind == "high":
        return u & np.uint64(0xFFFF000000000000)
    if kind == "low32":
        return u & np.uint64(0xFFFFFFFF)
    if kind == "and2":
        return u & uniform_keys64(n, seed + 1000)
    raise ValueError(f"unknown 64-bit key distribution {kind!r}")


def index_values(n: int, start: int = 0) -> np.ndarray:
    """Values equal to the original index: a stable sort keeps them rising
    within every run of equal keys."""
    return np.arange(start, start + n, dtype=np.uint64).astype(U32)


def and_keys(n: int, k: int, seed: int) -> np.ndarray:
    """Low-entropy keys: bitwise AND of k independent uniform words, so each
    bit is set with probability 2^-k."""
    rng = _rng(seed)
    out = np.full(n, 0xFFFFFFFF, dtype=U32)
    for _ in range(k):
        out &= rng.integers(0, 2**32, size=n, dtype=U32)
    return out


def top_byte_keys(n: int, top: int, seed: int) -> np.ndarray:
    """24 significant bits under a constant top byte."""
    low = _rng(seed).integers(0, 2**24, size=n, dtype=U32)
    return (U32(top & 0xFF) << U32(24)) | low


def zipf_probabilities(m: int = 16, s: float = 1.2) -> np.ndarray:
    ranks = np.arange(1, m + 1, dtype=np.float64)
    w = ranks ** (-s)
    return w / w.sum()


def zipf16_dictionary(seed: int, m: int = 16) -> np.ndarray:
    """m distinct u32 values drawn from the seed (duplicates rejected);
    entry r is the key of Zipf rank r + 1."""
    rng = _rng(seed)
    seen = []
    while len(seen) < m:
        x = int(rng.integers(0, 2**32, dtype=np.uint64))
        if x not in seen:
            seen.append(x)
    return np.array(seen, dtype=U32)


def zipf16_keys(n: int, seed: int, s: float = 1.2) -> np.ndarray:
    """Keys from a 16-entry dictionary with Zipf(s) rank frequencies."""
    d = zipf16_dictionary(seed)
    idx = _rng(seed + 1_000_003).choice(16, size=n, p=zipf_probabilities(16, s))
    return d[idx]


def batched_sizes(num_segments: int = 4096, lo_exp: float = 6.0, hi_exp: float = 20.0,
                  cap: int = 2**27, seed: int = SEED_BATCHED,
                  floor_size: int = 64) -> np.ndarray:
    """Segment sizes floor(2^u), u ~ U[lo_exp, hi_exp]; when the total runs
    past ``cap`` every size is scaled by cap/total (kept >= floor_size) and
    the largest segments are then trimmed until the total fits."""
    rng = _rng(seed)
    u = rng.uniform(lo_exp, hi_exp, size=num_segments)
    sizes = np.floor(np.exp2(u)).astype(np.int64)
    total = int(sizes.sum())
    if total > cap:
        sizes = np.maximum(floor_size, (sizes * cap) // total)
        total = int(sizes.sum())
        while total > cap:
            i = int(np.argmax(sizes))
            cut = min(total - cap, int(sizes[i]) - floor_size)
            if cut <= 0:
                raise ValueError("cap too small for the floor size")
            sizes[i] -= cut
            total -= cut
    return sizes.astype(U32)


def segment_offsets(sizes: np.ndarray) -> np.ndarray:
    """Exclusive running total of the sizes, with the grand total appended."""
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes.astype(np.uint64))
    if off[-1] > 0xFFFFFFFF:
        raise ValueError("segments exceed 2^32 - 1 items")
    return off.astype(U32)


def poisson_arrivals(rate_per_s: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: exponential gaps of mean 1/rate."""
    gaps = _rng(seed).exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


def serving_request_sizes(count: int, seed: int, lo_exp: float = 10.0,
                          hi_exp: float = 24.0) -> np.ndarray:
    """Request sizes floor(2^u), u ~ U[lo_exp, hi_exp]."""
    u = _rng(seed + 7).uniform(lo_exp, hi_exp, size=count)
    return np.floor(np.exp2(u)).astype(np.int64)


def serving_request_dists(count: int, seed: int) -> np.ndarray:
    """Key distribution per request, uniform over {uniform, AND-4, Zipf-16}."""
    return _rng(seed + 11).integers(0, 3, size=count).astype(np.int64)


# ---------------------------------------------------------------------------
# Counter-based (SplitMix64) generation, mirrored by the device generator.
# ---------------------------------------------------------------------------

def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (variant 13 of Stafford's mixers)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def splitmix64_words(state: int, first: int, count: int) -> np.ndarray:
    """Words first..first+count-1 of the SplitMix64 stream with this state."""
    i = np.arange(first, first + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state & MASK64) + (i + np.uint64(1)) * np.uint64(GOLDEN_GAMMA)
    return _mix64(z)


def stream_state(seed: int, stream_id: int) -> int:
    """State of request stream ``stream_id``: word ``stream_id`` of the
    SplitMix64 stream seeded with ``seed``."""
    return int(splitmix64_words(seed, stream_id, 1)[0])


def zipf16_thresholds(s: float = 1.2) -> np.ndarray:
    """Cumulative Zipf-16 probabilities as integers on the 2^32 scale; the
    last one is 2^32.  A draw u < t[r] (first such r) selects rank r + 1."""
    c = np.cumsum(zipf_probabilities(16, s))
    t = np.floor(c * 2.0**32).astype(np.uint64)
    t[-1] = np.uint64(2**32)
    return t


@dataclasses.dataclass(frozen=True)
class CounterGenParams:
    """Parameters of one device-generated request (shared with the library)."""
    dist: int
    state: int
    dictionary: Tuple[int, ...] = ()
    thresholds: Tuple[int, ...] = ()


def counter_params(dist: int, seed: int, stream_id: int) -> CounterGenParams:
    d = tuple(int(x) for x in zipf16_dictionary(seed)) if dist == DIST_ZIPF16 else ()
    t = tuple(int(x) for x in zipf16_thresholds()) if dist == DIST_ZIPF16 else ()
    return CounterGenParams(dist=dist, state=stream_state(seed, stream_id),
                            dictionary=d, thresholds=t)


def counter_keys(p: CounterGenParams, n: int, first: int = 0) -> np.ndarray:
    """Keys first..first+n-1 of a counter-generated request.

    uniform: low 32 bits of word i;
    AND-4:   AND of the two halves of words 2i and 2i+1;
    Zipf-16: the high 32 bits u of word i pick the first rank r with
             u < thresholds[r]; the key is dictionary[r].
    """
    if p.dist == DIST_UNIFORM:
        w = splitmix64_words(p.state, first, n)
        return (w & np.uint64(0xFFFFFFFF)).astype(U32)
    if p.dist == DIST_AND4:
        w = splitmix64_words(p.state, 2 * first, 2 * n).reshape(n, 2)
        lo = w & np.uint64(0xFFFFFFFF)
        hi = w >> np.uint64(32)
        r = lo[:, 0] & hi[:, 0] & lo[:, 1] & hi[:, 1]
        return r.astype(U32)
    if p.dist == DIST_ZIPF16:
        w = splitmix64_words(p.state, first, n)
        u = w >> np.uint64(32)
        t = np.array(p.thresholds, dtype=np.uint64)
        r = np.searchsorted(t, u, side="right")
        return np.array(p.dictionary, dtype=U32)[r]
    raise ValueError(f"unknown distribution id {p.dist}")


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    with_values: bool
    kind: str                 # uniform | and | top_byte | zipf16
    seed: int
    param: int = 0            # k for AND-of-k, the top byte for top_byte
    key_bits: int = 32        # 64: u64 keys (kind as in keys64)


WORKLOADS: Dict[str, Workload] = {
    "keys_1m_uniform": Workload("keys_1m_uniform", 2**20, False, "uniform", SEED_KEYS_1M),
    "pairs_256m_uniform": Workload("pairs_256m_uniform", 2**28, True, "uniform", SEED_PAIRS_256M),
    "keys_256m_uniform": Workload("keys_256m_uniform", 2**28, False, "uniform", SEED_KEYS_256M),
    "pairs_64m_and2": Workload("pairs_64m_and2", 2**26, True, "and", SEED_AND[2], 2),
    "pairs_64m_and4": Workload("pairs_64m_and4", 2**26, True, "and", SEED_AND[4], 4),
    "pairs_64m_and8": Workload("pairs_64m_and8", 2**26, True, "and", SEED_AND[8], 8),
    "pairs_64m_top_a5": Workload("pairs_64m_top_a5", 2**26, True, "top_byte", SEED_TOP_BYTE, 0xA5),
    "pairs_64m_zipf16": Workload("pairs_64m_zipf16", 2**26, True, "zipf16", SEED_ZIPF16),
    "keys_64m_uniform": Workload("keys_64m_uniform", 2**26, False, "uniform", SEED_TABLE1),
    "pairs_64m_uniform": Workload("pairs_64m_uniform", 2**26, True, "uniform", SEED_TABLE1),
    "pairs64_256m_uniform": Workload("pairs64_256m_uniform", 2**28, True, "uniform", SEED_PAIRS64_256M,
                                     key_bits=64),
}


def make_keys(kind: str, n: int, seed: int, param: int = 0) -> np.ndarray:
    if kind == "uniform":
        return uniform_keys(n, seed)
    if kind == "and":
        return and_keys(n, param, seed)
    if kind == "top_byte":
        return top_byte_keys(n, param, seed)
    if kind == "zipf16":
        return zipf16_keys(n, seed)
    raise ValueError(f"unknown key distribution {kind!r}")


def make_workload(w: Workload, n: Optional[int] = None):
    """(keys, values-or-None) for a named workload, optionally at a smaller n
    with the same distribution and seed."""
    n = w.n if n is None else n
    keys = keys64(w.kind, n, w.seed) if w.key_bits == 64 else make_keys(w.kind, n, w.seed, w.param)
    vals = index_values(n) if w.with_values else None
    return keys, vals
