"""Parity of the HIP sort with the CPU oracle: bit-exact, on seeded inputs.

Sizes span one to many tiles with ragged tails; the distributions are the
skewed workloads (low-entropy AND-of-k keys, constant top byte, 16-key Zipf)
plus sorted, reversed and all-equal arrays; every digit decomposition and
tile shape the library compiles is exercised.  Values are original indices,
so any instability or lost item shows up as a value mismatch.
"""
import numpy as np
import pytest

import oracle
import paper_1008_2849_amd as rts
from paper_1008_2849_amd import inputs
from paper_1008_2849_amd.api import (Config, FLAG_CHUNKS, FLAG_DIRECT_SCATTER, FLAG_NO_SKIP, FLAG_NT_STORES,
                                     FLAG_ONE_CHAIN)
from gpu_util import announce, sync, to_dev, to_host

pytestmark = pytest.mark.gpu

TILE = 1024 * 16  # the default tile
SIZES = [0, 1, 2, 3, 63, 64, 65, 1000, TILE - 1, TILE, TILE + 1, 3 * TILE + 77, 100_003,
         (1 << 20) - 1, 1 << 20, (1 << 20) + 1]


def gpu_sort(keys, vals=None, cfg=None):
    k = to_dev(keys)
    v = None if vals is None else to_dev(vals)
    if cfg is None:
        if v is None:
            rts.sort_keys(k)
        else:
            rts.sort_pairs(k, v)
    else:
        rts.sort_ex(k, v, cfg)
    sync()
    return to_host(k), (None if v is None else to_host(v))


def assert_same(got, want, what=""):
    gk, gv = got
    wk, wv = want
    assert gk.shape == wk.shape, what
    if not np.array_equal(gk, wk):
        bad = np.nonzero(gk != wk)[0]
        raise AssertionError(f"{what}: keys differ at {bad.size} positions, first {bad[:5]}")
    if wv is not None:
        if not np.array_equal(gv, wv):
            bad = np.nonzero(gv != wv)[0]
            raise AssertionError(f"{what}: values differ at {bad.size} positions, first {bad[:5]}")


@pytest.mark.parametrize("n", SIZES)
def test_pairs_uniform_sizes(n):
    announce(f"pairs uniform n={n}")
    k = inputs.uniform_keys(n, 100 + n % 997)
    v = inputs.index_values(n)
    assert_same(gpu_sort(k, v), oracle.lsd_sort(k, v), f"n={n}")


@pytest.mark.parametrize("n", SIZES)
def test_keys_uniform_sizes(n):
    announce(f"keys uniform n={n}")
    k = inputs.uniform_keys(n, 200 + n % 991)
    assert_same(gpu_sort(k), oracle.lsd_sort(k), f"n={n}")


def _dist_cases(n):
    idx = np.arange(n, dtype=np.uint32)
    return {
        "and2": inputs.and_keys(n, 2, 31),
        "and4": inputs.and_keys(n, 4, 32),
        "and8": inputs.and_keys(n, 8, 33),
        "top_a5": inputs.top_byte_keys(n, 0xA5, 34),
        "top_00": inputs.top_byte_keys(n, 0x00, 36),
        "zipf16": inputs.zipf16_keys(n, 35),
        "all_equal": np.full(n, 0x12345678, dtype=np.uint32),
        "all_zero": np.zeros(n, dtype=np.uint32),
        "all_ones": np.full(n, 0xFFFFFFFF, dtype=np.uint32),
        "sorted": idx,
        "reversed": idx[::-1].copy(),
        "two_values": np.where(inputs.uniform_keys(n, 37) & 1, 0xFFFFFFFF, 0).astype(np.uint32),
        "low_byte_only": (inputs.uniform_keys(n, 38) & 0xFF).astype(np.uint32),
    }


@pytest.mark.parametrize("dist", list(_dist_cases(8).keys()))
def test_distributions_pairs(dist):
    n = (1 << 20) + 123
    announce(f"pairs dist={dist} n={n}")
    k = _dist_cases(n)[dist]
    v = inputs.index_values(n)
    assert_same(gpu_sort(k, v), oracle.lsd_sort(k, v), dist)


@pytest.mark.parametrize("dist", ["and8", "top_a5", "zipf16", "all_equal"])
def test_distributions_keys(dist):
    n = (1 << 19) + 5
    announce(f"keys dist={dist} n={n}")
    k = _dist_cases(n)[dist]
    assert_same(gpu_sort(k), oracle.lsd_sort(k), dist)


WIDTHS = [(8, 8, 8, 8), (11, 11, 10), (10, 11, 11), (4,) * 8, (6, 6, 6, 6, 8), (11, 8, 8, 5),
          (8, 8, 8, 4, 4), (11, 11, 6, 4)]
SHAPES = [(256, 16), (512, 16), (1024, 8), (1024, 16), (512, 32)]
SHAPES_WIDE = {(256, 16), (512, 8), (512, 16)}  # shapes built for 9..11-bit digits


@pytest.mark.parametrize("widths", WIDTHS, ids=["-".join(map(str, w)) for w in WIDTHS])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{b}x{i}" for b, i in SHAPES])
def test_configs(widths, shape):
    n = 300_001
    announce(f"config widths={widths} shape={shape} n={n}")
    k = inputs.and_keys(n, 2, 7)
    v = inputs.index_values(n)
    cfg = Config(widths, shape[0], shape[1], 0)
    if max(widths) > 8 and shape not in SHAPES_WIDE:
        # larger tiles need more LDS than a CU has once digits exceed 8 bits;
        # the library declines the shape instead of failing the launch
        with pytest.raises(rts.RtError) as e:
            gpu_sort(k, v, cfg)
        assert e.value.status == 6
        return
    assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v, widths), f"{widths} {shape}")


@pytest.mark.parametrize("n", [2, 1000, 16383, 16384, 16385, 5 * 16384 + 77, 1_000_003, (1 << 25) + 77])
def test_two_blocks_per_cu_shape(n):
    """512 x 32 tiles (16K items; the values staged after the keys leave,
    so two blocks share a CU): pairs and keys only, uniform and skewed keys,
    forced XCD chunks, one chain and the probed default, each the oracle's."""
    announce(f"512x32 n={n}")
    v = inputs.index_values(n)
    flag_sets = (0, FLAG_CHUNKS, FLAG_ONE_CHAIN | FLAG_NO_SKIP) if n < (1 << 25) else (0,)
    for dist in ("uniform", "and4", "top_a5"):
        k = inputs.uniform_keys(n, 95) if dist == "uniform" else _dist_cases(n)[dist]
        want_kv = oracle.lsd_sort(k, v)
        want_k = want_kv[0]
        for flags in flag_sets:
            cfg = Config((8, 8, 8, 8), 512, 32, flags)
            assert_same(gpu_sort(k, v, cfg), want_kv, f"pairs {dist} flags={flags}")
            assert_same(gpu_sort(k, None, cfg), (want_k, None), f"keys {dist} flags={flags}")


@pytest.mark.parametrize("flags", [FLAG_NO_SKIP, FLAG_NT_STORES, FLAG_NO_SKIP | FLAG_NT_STORES,
                                   FLAG_DIRECT_SCATTER, FLAG_DIRECT_SCATTER | FLAG_NO_SKIP])
@pytest.mark.parametrize("dist", ["top_a5", "low_byte_only", "all_equal", "and4"])
def test_flags(flags, dist):
    n = 200_017
    announce(f"flags={flags} dist={dist} n={n}")
    k = _dist_cases(n)[dist]
    v = inputs.index_values(n)
    cfg = Config((8, 8, 8, 8), 1024, 16, flags)
    assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v), f"flags={flags} {dist}")
    assert_same(gpu_sort(k, None, cfg), oracle.lsd_sort(k), f"keys flags={flags} {dist}")


@pytest.mark.parametrize("n", [100_003, 3 * TILE * 8 + 77])
def test_validated_sort(n):
    """RT_FLAG_VALIDATE waits for the sort and reads its device error word:
    a correct sort returns RT_OK (no exception) with the oracle's result,
    through the library's workspace and a caller workspace, in XCD chunks
    and on one chain."""
    import torch
    from paper_1008_2849_amd.api import FLAG_VALIDATE
    announce(f"validated sort n={n}")
    k = inputs.uniform_keys(n, 91)
    v = inputs.index_values(n)
    want = oracle.lsd_sort(k, v)
    for extra in (FLAG_CHUNKS, FLAG_ONE_CHAIN):
        cfg = Config((8, 8, 8, 8), 1024, 16, FLAG_VALIDATE | extra)
        assert_same(gpu_sort(k, v, cfg), want, f"validate {extra}")
        kd, vd = to_dev(k), to_dev(v)
        ws = torch.empty(rts.workspace_bytes(n, True, cfg), dtype=torch.uint8, device="cuda")
        rts.sort_ex(kd, vd, cfg, ws)
        assert_same((to_host(kd), to_host(vd)), want, f"validate {extra} caller workspace")


@pytest.mark.parametrize("n,dist", [(1000, "uniform"), (3 * TILE + 77, "uniform"), (3 * TILE + 77, "and4"),
                                    ((1 << 22) + 123, "uniform"), ((1 << 22) + 123, "zipf16")])
def test_fused_histogram(n, dist):
    """RT_FLAG_FUSED_HISTOGRAM: passes 0-2 count the next pass's digit while
    they write, and the sort still equals the oracle's, pairs and keys only,
    with ragged last tiles, under 8x4 digits, two 4-bit digits in other
    shapes, and 4-bit digits throughout."""
    from paper_1008_2849_amd.api import FLAG_FUSED_HISTOGRAM
    announce(f"fused histogram n={n} dist={dist}")
    k = inputs.uniform_keys(n, 94) if dist == "uniform" else _dist_cases(n)[dist]
    v = inputs.index_values(n)
    for widths, shape in (((8, 8, 8, 8), (1024, 16)), ((4, 4, 8, 8, 8), (512, 16)), ((4,) * 8, (1024, 8))):
        cfg = Config(widths, shape[0], shape[1], FLAG_FUSED_HISTOGRAM)
        assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v, widths), f"fused {widths}")
        assert_same(gpu_sort(k, None, cfg), oracle.lsd_sort(k, None, widths), f"fused keys {widths}")


@pytest.mark.parametrize("widths,shape", [((11, 11, 10), (512, 16)), ((8, 8, 8, 8), (256, 16)),
                                          ((4,) * 8, (1024, 8))])
def test_direct_scatter_configs(widths, shape):
    """The pass without LDS staging gives the same result under other digit
    widths and tile shapes, with a ragged last tile."""
    n = 7 * shape[0] * shape[1] + 4321
    announce(f"direct scatter widths={widths} shape={shape} n={n}")
    k = inputs.and_keys(n, 2, 17)
    v = inputs.index_values(n)
    cfg = Config(widths, shape[0], shape[1], FLAG_DIRECT_SCATTER)
    assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v, widths), f"{widths} {shape}")
    assert_same(gpu_sort(k, None, cfg), oracle.lsd_sort(k, None, widths), f"keys {widths} {shape}")


@pytest.mark.parametrize("dist", list(_dist_cases(8).keys()))
def test_chunk_flags(dist):
    """XCD chunks forced at a size below the default's threshold, and one
    lookback chain per pass, both give the oracle's result, with and without
    pass skipping, keys only and pairs."""
    n = 3 * TILE * 8 + 999
    announce(f"chunk flags dist={dist} n={n}")
    k = _dist_cases(n)[dist]
    v = inputs.index_values(n)
    for flags in (FLAG_CHUNKS, FLAG_CHUNKS | FLAG_NO_SKIP, FLAG_ONE_CHAIN, FLAG_ONE_CHAIN | FLAG_NO_SKIP):
        cfg = Config((8, 8, 8, 8), 1024, 16, flags)
        assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v), f"flags={flags} {dist}")
    cfg = Config((8, 8, 8, 8), 1024, 16, FLAG_CHUNKS)
    assert_same(gpu_sort(k, None, cfg), oracle.lsd_sort(k), f"keys chunks {dist}")


# The sample's decision where it is clear from the distribution: uniform and
# constant-top-byte keys balance the chunks; AND-4 keys (digit 0 in 60 % of
# them) and Zipf-16 keys (the first key in about 36 %) put far more than
# 1/64 of the sample in one bin.  None: not asserted.
PROBE_EXPECTED = {"uniform": 1, "top_a5": 1, "and4": 0, "zipf16": 0, "low_byte_only": None, "sorted": None}


@pytest.mark.parametrize("dist", list(PROBE_EXPECTED))
def test_probed_sizes(dist):
    """At 2^25 items and above the default samples the keys and picks XCD
    chunks (uniform, constant top byte) or one chain (skewed keys): the
    decision is the expected one, and the result is the oracle's either
    way."""
    import torch
    n = (1 << 25) + 77
    announce(f"probed dist={dist} n={n}")
    k = inputs.uniform_keys(n, 700) if dist == "uniform" else _dist_cases(n)[dist]
    v = inputs.index_values(n)
    mode = rts.chunk_decision(torch.from_numpy(k.view(np.int32)).cuda())
    assert mode in (0, 1)
    if PROBE_EXPECTED[dist] is not None:
        assert mode == PROBE_EXPECTED[dist], f"{dist}: chunk decision {mode}"
    assert_same(gpu_sort(k, v), oracle.lsd_sort(k, v), dist)


def test_chunk_decision_fixed_cases():
    """Where no sample is taken the decision follows the size, the digit
    widths and the flags: below 2^25 items one chain, RT_FLAG_CHUNKS chunks at
    any size, RT_FLAG_ONE_CHAIN and 11-bit digits one chain."""
    import torch
    announce("chunk decision fixed cases")
    small = torch.from_numpy(inputs.uniform_keys(1 << 20, 701).view(np.int32)).cuda()
    assert rts.chunk_decision(small) == 0
    assert rts.chunk_decision(small[:1]) == 0
    assert rts.chunk_decision(small, cfg=Config((8, 8, 8, 8), 1024, 16, FLAG_CHUNKS)) == 1
    big = torch.from_numpy(_dist_cases((1 << 25) + 1)["and4"].view(np.int32)).cuda()
    assert rts.chunk_decision(big, cfg=Config((8, 8, 8, 8), 1024, 16, FLAG_CHUNKS)) == 1
    assert rts.chunk_decision(big, cfg=Config((8, 8, 8, 8), 1024, 16, FLAG_ONE_CHAIN)) == 0
    assert rts.chunk_decision(big, cfg=Config((11, 11, 10), 512, 16, 0)) == 0


def test_probed_keys_only_tuned_shape():
    """Keys only at 2^25 items with the tuned shape (512 x 32 tiles, two
    blocks per CU) in XCD chunks: the oracle's result."""
    rts.load_default_tuning()
    n = (1 << 25) + 5
    announce(f"probed keys only n={n}")
    k = inputs.uniform_keys(n, 703)
    assert_same(gpu_sort(k), oracle.lsd_sort(k), "keys only")


@pytest.mark.parametrize("skip_pattern", [1, 2, 5, 6, 9, 14])
def test_chunks_with_skipped_passes(skip_pattern):
    """A skipped pass (constant digit) leaves the next pass a single chunk:
    its chunks come from the skipped digit's ranges."""
    n = 40 * TILE + 5
    announce(f"chunks skip pattern {skip_pattern:04b} n={n}")
    k = inputs.uniform_keys(n, 600 + skip_pattern)
    for p in range(4):
        if skip_pattern >> p & 1:
            k = (k & ~np.uint32(0xFF << (8 * p))) | np.uint32((0x3C + p) << (8 * p))
    v = inputs.index_values(n)
    cfg = Config((8, 8, 8, 8), 1024, 16, FLAG_CHUNKS)
    assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v), f"pattern {skip_pattern}")


CHUNK_WIDTHS = [(1, 2, 3, 8, 8, 5, 5), (3, 3, 3, 3, 4, 8, 8), (8, 1, 7, 8, 8), (2, 6, 8, 8, 8)]


@pytest.mark.parametrize("widths", CHUNK_WIDTHS, ids=["-".join(map(str, w)) for w in CHUNK_WIDTHS])
@pytest.mark.parametrize("dist", ["uniform", "and2", "zipf16"])
def test_chunks_narrow_digits(widths, dist):
    """Digits narrower than 3 bits give their successor pass fewer than 8
    chunks (one per digit value); the chunks of every pass still tile its
    input once."""
    n = 9 * 512 * 16 + 321
    announce(f"chunks widths={widths} dist={dist} n={n}")
    k = inputs.uniform_keys(n, 77) if dist == "uniform" else _dist_cases(n)[dist]
    v = inputs.index_values(n)
    cfg = Config(widths, 512, 16, FLAG_CHUNKS)
    assert_same(gpu_sort(k, v, cfg), oracle.lsd_sort(k, v, widths), f"{widths} {dist}")
    assert_same(gpu_sort(k, None, cfg), oracle.lsd_sort(k, None, widths), f"keys {widths} {dist}")


@pytest.mark.parametrize("n", [2, 1000, TILE - 1, TILE * 5 + 3, TILE * 8 - 1, TILE * 8, TILE * 8 + 1, TILE * 9 + 5,
                               TILE * 15, TILE * 23 + 4097])
def test_chunk_bounds_first_pass(n):
    """Sizes around multiples of 8 tiles: the first pass's chunks by position
    have equal or unequal tile counts, empty ones included for small n."""
    announce(f"chunk bounds n={n}")
    k = inputs.uniform_keys(n, 500 + n % 101)
    v = inputs.index_values(n)
    assert_same(gpu_sort(k, v, Config((8, 8, 8, 8), 1024, 16, FLAG_CHUNKS)), oracle.lsd_sort(k, v), f"n={n}")
    assert_same(gpu_sort(k, v, Config((8, 8, 8, 8), 256, 16, FLAG_CHUNKS)), oracle.lsd_sort(k, v), f"4K n={n}")


@pytest.mark.parametrize("skip_pattern", range(16))
def test_every_executed_pass_count(skip_pattern):
    # byte p of every key is constant when bit p of skip_pattern is set, so
    # each subset of passes (0..4 executed) is covered, odd counts included.
    n = 50_000 + skip_pattern
    announce(f"skip pattern {skip_pattern:04b} n={n}")
    k = inputs.uniform_keys(n, 300 + skip_pattern)
    for p in range(4):
        if skip_pattern >> p & 1:
            k = (k & ~np.uint32(0xFF << (8 * p))) | np.uint32((0x5A + p) << (8 * p))
    v = inputs.index_values(n)
    assert_same(gpu_sort(k, v), oracle.lsd_sort(k, v), f"pattern {skip_pattern}")
    assert_same(gpu_sort(k), oracle.lsd_sort(k), f"keys pattern {skip_pattern}")


def test_unaligned_views():
    import torch
    n = 123_457
    for off in (1, 2, 3):
        announce(f"unaligned view offset {off}")
        k = inputs.uniform_keys(n, 40 + off)
        v = inputs.index_values(n)
        kb = to_dev(np.concatenate([np.zeros(off, np.uint32), k, np.zeros(5, np.uint32)]))
        vb = to_dev(np.concatenate([np.zeros(off + 2, np.uint32), v, np.zeros(5, np.uint32)]))
        kv, vv = kb[off:off + n], vb[off + 2:off + 2 + n]
        rts.sort_pairs(kv, vv)
        torch.cuda.synchronize()
        got = (to_host(kv), to_host(vv))
        assert_same(got, oracle.lsd_sort(k, v), f"offset {off}")
        # guard words around the views are untouched
        assert np.all(to_host(kb[:off]) == 0) and np.all(to_host(kb[off + n:]) == 0)
        assert np.all(to_host(vb[:off + 2]) == 0) and np.all(to_host(vb[off + 2 + n:]) == 0)


def test_histograms_match_oracle():
    n = 1_000_003
    k = inputs.and_keys(n, 2, 50)
    for widths in [(8, 8, 8, 8), (11, 11, 10), (4,) * 8]:
        announce(f"histograms {widths}")
        h = rts.digit_histograms(to_dev(k), Config(widths, 256, 16))
        sync()
        h = h.cpu().numpy().view(np.uint32)
        shift = 0
        for p, w in enumerate(widths):
            want = oracle.digit_histogram(k, shift, w)
            assert np.array_equal(h[p, :1 << w].astype(np.uint64), want), (widths, p)
            shift += w


@pytest.mark.parametrize("shift,width", [(0, 8), (8, 8), (24, 8), (0, 11), (11, 11), (22, 10), (28, 4), (31, 1)])
def test_single_counting_pass(shift, width):
    import torch
    n = 777_777
    announce(f"counting pass shift={shift} width={width}")
    k = inputs.uniform_keys(n, 60 + shift)
    v = inputs.index_values(n)
    kin, vin = to_dev(k), to_dev(v)
    kout, vout = torch.empty_like(kin), torch.empty_like(vin)
    rts.counting_pass(kin, vin, kout, vout, shift, width)
    sync()
    want = oracle.counting_pass(k, v, shift, width)
    assert_same((to_host(kout), to_host(vout)), want, f"pass {shift}/{width}")
    assert np.array_equal(to_host(kin), k)  # input untouched


def test_repeat_is_deterministic():
    n = (1 << 22) + 3
    announce(f"determinism x20 n={n}")
    k = inputs.uniform_keys(n, 70)
    v = inputs.index_values(n)
    want = oracle.lsd_sort(k, v)
    import torch
    kd0, vd0 = to_dev(k), to_dev(v)
    for it in range(20):
        kd, vd = kd0.clone(), vd0.clone()
        rts.sort_pairs(kd, vd)
        torch.cuda.synchronize()
        assert_same((to_host(kd), to_host(vd)), want, f"repeat {it}")


def test_explicit_workspace_and_streams():
    import torch
    n = 500_000
    announce("explicit workspace, two streams")
    cfg = Config((8, 8, 8, 8), 256, 16, 0)
    need = rts.workspace_bytes(n, True, cfg)
    assert need > 0
    small = torch.empty(need // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(rts.RtError):
        rts.sort_ex(to_dev(np.arange(n, dtype=np.uint32)), to_dev(np.arange(n, dtype=np.uint32)), cfg, small)
    cases = []
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for i, s in enumerate(streams):
        k = inputs.uniform_keys(n, 80 + i)
        v = inputs.index_values(n)
        kd, vd = to_dev(k), to_dev(v)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        rts.sort_ex(kd, vd, cfg, ws, stream=s)
        cases.append((k, v, kd, vd, ws))
    torch.cuda.synchronize()
    for k, v, kd, vd, _ in cases:
        assert_same((to_host(kd), to_host(vd)), oracle.lsd_sort(k, v), "stream case")


def test_generator_matches_host_definition():
    import torch
    n = 300_000
    for dist in (inputs.DIST_UNIFORM, inputs.DIST_AND4, inputs.DIST_ZIPF16):
        announce(f"generator dist={dist}")
        p = inputs.counter_params(dist, 5, 17 + dist)
        kd = torch.empty(n, dtype=torch.int32, device="cuda")
        vd = torch.empty(n, dtype=torch.int32, device="cuda")
        rts.generate(kd, vd, p, value_base=1000)
        sync()
        assert np.array_equal(to_host(kd), inputs.counter_keys(p, n))
        assert np.array_equal(to_host(vd), np.arange(1000, 1000 + n, dtype=np.uint32))


def test_copy_probe():
    import torch
    n = (1 << 20) + 3
    a = to_dev(inputs.uniform_keys(n, 90))
    b = torch.zeros_like(a)
    rts.copy(a, b)
    sync()
    assert torch.equal(a, b)
    c = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
    rts.copy(a[1:], c[1:n])  # not 16-byte aligned
    sync()
    assert torch.equal(c[1:n], a[1:])


def test_bandwidth_probes():
    """The probes move what they say: both copies reproduce the source, the
    write probe writes its pattern (word i: i, 1, 2, 3), the read probe
    leaves its source alone."""
    import torch
    from paper_1008_2849_amd import _lib
    n = (1 << 22) + 64  # 16-byte words: a multiple of 4 items, past one grid stride
    a = to_dev(inputs.uniform_keys(n, 93))
    for kind in (_lib.RT_PROBE_COPY, _lib.RT_PROBE_COPY_NT):
        b = torch.zeros_like(a)
        rts.bandwidth_probe(kind, src=a, dst=b)
        sync()
        assert torch.equal(a, b), kind
    w = torch.zeros_like(a)
    rts.bandwidth_probe(_lib.RT_PROBE_WRITE, dst=w)
    sync()
    words = w.view(-1, 4).cpu().numpy().view(np.uint32)
    assert np.array_equal(words[:, 0], np.arange(n // 4, dtype=np.uint32))
    assert (words[:, 1:] == np.array([1, 2, 3], dtype=np.uint32)).all()
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    before = a.clone()
    rts.bandwidth_probe(_lib.RT_PROBE_READ, src=a, sink=sink)
    sync()
    assert torch.equal(a, before)


@pytest.mark.parametrize("n,dist", [(3 * TILE + 1234, "uniform"), ((1 << 25) + 1234, "uniform"),
                                    ((1 << 25) + 1234, "and4")])
def test_graph_capture_single_sort_replays(n, dist):
    """rt_sort_pairs_ex with a caller workspace only enqueues kernels: captured
    once into a graph, each replay sorts its fresh input like the eager call
    (fills are kernels, never memsets, so replays after the first are sound).
    At 2^25 items the probe and the XCD chunks (uniform) or one chain (AND-4)
    run inside the graph too."""
    import torch
    announce(f"graph capture single sort n={n} {dist}")
    k_h = inputs.uniform_keys(n, 81) if dist == "uniform" else inputs.and_keys(n, 4, 82)
    v_h = inputs.index_values(n)
    want = oracle.lsd_sort(k_h, v_h)
    k0, v0 = to_dev(k_h), to_dev(v_h)
    k, v = k0.clone(), v0.clone()
    cfg = Config((8, 8, 8, 8), 1024, 16, 0)
    ws = torch.empty(rts.workspace_bytes(n, True, cfg), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rts.sort_ex(k, v, cfg, ws, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    sync()
    assert_same((to_host(k), to_host(v)), want, "eager")
    g = torch.cuda.CUDAGraph()
    k.copy_(k0)
    v.copy_(v0)
    sync()
    with torch.cuda.graph(g, stream=s):
        rts.sort_ex(k, v, cfg, ws, stream=s)
    for rep in range(3):
        k.copy_(k0)
        v.copy_(v0)
        sync()
        g.replay()
        sync()
        assert_same((to_host(k), to_host(v)), want, f"replay {rep}")
        k2, v2 = k0.clone(), v0.clone()
        rts.sort_pairs(k2, v2)
        sync()
        assert_same((to_host(k2), to_host(v2)), want, f"eager after replay {rep}")


@pytest.mark.parametrize("name", ["pairs_64m_and2", "pairs_64m_and4", "pairs_64m_and8", "pairs_64m_top_a5",
                                  "pairs_64m_zipf16"])
def test_skewed_workloads_full_size(name):
    """The skewed workloads at their full 2^26-pair size, with the tuned
    configuration the benchmark uses, bit-exact against the oracle."""
    w = inputs.WORKLOADS[name]
    announce(f"full-size workload {name} n={w.n}")
    k, v = inputs.make_workload(w)
    assert_same(gpu_sort(k, v), oracle.lsd_sort(k, v), name)


def test_keys_1m_workload_tuned():
    """The 2^20 keys-only workload with the autotuned table loaded."""
    import os
    from paper_1008_2849_amd import _lib
    w = inputs.WORKLOADS["keys_1m_uniform"]
    announce(f"keys workload n={w.n} tuned")
    rts.load_tuning(_lib.TUNING_PATH if os.path.exists(_lib.TUNING_PATH) else None)
    try:
        k, _ = inputs.make_workload(w)
        assert_same(gpu_sort(k), oracle.lsd_sort(k), "keys_1m")
    finally:
        rts.load_default_tuning()
