"""Parity of the batched segmented sort with the CPU oracle, bit-exact.

Segment sizes straddle every size-class boundary of the library (the
whole-in-LDS classes up to 2048, 8192 and 16384 items, and the tiled path
beyond) and include empty and one-item segments; the batched workload's
log-uniform size mix is tested at a reduced total and, at its full 2^27
total, on sampled segments.  Values are global original indices, so an item
that leaves its segment, is lost or breaks stability shows up as a value
mismatch.
"""
import numpy as np
import pytest

import oracle
import paper_1008_2849_amd as rts
from paper_1008_2849_amd import inputs
from paper_1008_2849_amd._lib import RtError, RT_ERR_INVALID_ARG
from gpu_util import announce, sync, to_dev, to_host

pytestmark = pytest.mark.gpu

BOUNDARY_SIZES = [0, 1, 2, 3, 63, 64, 65, 2047, 2048, 2049, 5000, 8191, 8192, 8193, 12000, 16383, 16384,
                  16385, 16384 * 2, 16384 * 3 + 1, 40000, 100_003]


def offsets_of(sizes, start=0):
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(np.asarray(sizes, dtype=np.uint64))
    return (off + start).astype(np.uint32)


def run_batched(keys, vals, off, max_total=None, validate=False, ex=False):
    k = to_dev(keys)
    v = None if vals is None else to_dev(vals)
    o = to_dev(off)
    total = int(off[-1]) - int(off[0]) if max_total is None else max_total
    if ex or validate:
        rts.sort_batched_ex(k, v, o, total, validate=validate)
    else:
        rts.sort_pairs_batched(k, v, o, total)
    sync()
    return to_host(k), (None if v is None else to_host(v))


def check(got, want, what):
    gk, gv = got
    wk, wv = want
    if not np.array_equal(gk, wk):
        bad = np.nonzero(gk != wk)[0]
        raise AssertionError(f"{what}: keys differ at {bad.size} positions, first {bad[:5]}")
    if wv is not None and not np.array_equal(gv, wv):
        bad = np.nonzero(gv != wv)[0]
        raise AssertionError(f"{what}: values differ at {bad.size} positions, first {bad[:5]}")


@pytest.mark.parametrize("with_values", [True, False])
@pytest.mark.parametrize("seed", [1, 2])
def test_boundary_sizes(with_values, seed):
    rng = np.random.default_rng(seed)
    sizes = list(BOUNDARY_SIZES)
    rng.shuffle(sizes)
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched boundary sizes seed={seed} values={with_values} n={n} segments={len(sizes)}")
    k = inputs.uniform_keys(n, 500 + seed)
    v = inputs.index_values(n) if with_values else None
    check(run_batched(k, v, off), oracle.lsd_sort_segmented(k, v, off), "boundary sizes")


@pytest.mark.parametrize("kind", ["and4", "and8", "zipf16", "top_a5", "all_equal", "sorted", "reversed"])
def test_skewed_segments(kind):
    sizes = [3000, 16384, 20000, 70000, 5, 9000]
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched skewed {kind} n={n}")
    keys = {
        "and4": lambda: inputs.and_keys(n, 4, 32),
        "and8": lambda: inputs.and_keys(n, 8, 33),
        "zipf16": lambda: inputs.zipf16_keys(n, 35),
        "top_a5": lambda: inputs.top_byte_keys(n, 0xA5, 34),
        "all_equal": lambda: np.full(n, 7, dtype=np.uint32),
        "sorted": lambda: np.arange(n, dtype=np.uint32),
        "reversed": lambda: np.arange(n, dtype=np.uint32)[::-1].copy(),
    }[kind]()
    v = inputs.index_values(n)
    check(run_batched(keys, v, off), oracle.lsd_sort_segmented(keys, v, off), kind)


@pytest.mark.parametrize("kind", ["uniform", "and4"])
def test_long_segments_in_xcd_chunks(kind):
    """At least 128 segments of at least 16 tiles on average: the tiled
    passes split the tile list into XCD chunks at segment ends, with
    segments of uneven length (a few much longer ones) and a one-item and an
    empty segment among them."""
    rng = np.random.default_rng(7)
    sizes = [int(x) for x in rng.integers(200_000, 400_000, size=136)]
    sizes[5] = 2_000_003   # one long segment: chunks of uneven tile counts
    sizes[70] = 1
    sizes[71] = 0
    sizes[100] = 16384 * 16
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched XCD chunks {kind} segments={len(sizes)} n={n}")
    k = inputs.uniform_keys(n, 900) if kind == "uniform" else inputs.and_keys(n, 4, 901)
    v = inputs.index_values(n)
    check(run_batched(k, v, off), oracle.lsd_sort_segmented(k, v, off), kind)


def test_batched_workload_mix_reduced():
    """The batched workload's size mix (log-uniform 2^6..2^20, capped) at a
    2^22 total, so the oracle checks every segment."""
    sizes = inputs.batched_sizes(num_segments=512, cap=1 << 22)
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched mix 512 segments n={n}")
    k = inputs.uniform_keys(n, inputs.SEED_BATCHED)
    v = inputs.index_values(n)
    check(run_batched(k, v, off), oracle.lsd_sort_segmented(k, v, off), "mix")


def test_batched_workload_full_size_sampled():
    """4096 segments totalling 2^27 pairs (the measured batched workload, in
    the launch configuration the benchmark times); the oracle sorts a sample
    of the segments one by one, every other segment is checked by the
    properties that fix a stable sort of original indices."""
    import torch
    sizes = inputs.batched_sizes()
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched full workload 4096 segments n={n}")
    k_h = inputs.uniform_keys(n, inputs.SEED_BATCHED)
    k = to_dev(k_h)
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    o = to_dev(off)
    rts.sort_pairs_batched(k, v, o, n)
    sync()
    gk, gv = to_host(k), to_host(v)
    rng = np.random.default_rng(9)
    big = np.argsort(sizes)[-4:]  # the largest segments
    pick = np.unique(np.concatenate([big, rng.choice(len(sizes), 24, replace=False)]))
    for s in pick:
        a, b = int(off[s]), int(off[s + 1])
        wk, wv = oracle.lsd_sort(k_h[a:b], np.arange(a, b, dtype=np.uint32))
        assert np.array_equal(gk[a:b], wk) and np.array_equal(gv[a:b], wv), f"segment {s} [{a},{b})"
    # every segment: values are a permutation of its own index range, keys
    # ascend, equal keys keep index order, and each key came with its index
    seg = np.repeat(np.arange(len(sizes)), sizes)
    assert np.all(np.bincount(gv, minlength=n) == 1)
    assert np.array_equal(seg[gv], seg)
    assert np.array_equal(k_h[gv], gk)
    same_seg = seg[1:] == seg[:-1]
    kk = gk.astype(np.uint64)
    assert np.all(kk[1:][same_seg] >= kk[:-1][same_seg])
    eq = same_seg & (gk[1:] == gk[:-1])
    assert np.all(gv[1:][eq] > gv[:-1][eq])


def test_untouched_outside_and_offset_start():
    """off[0] > 0: items before off[0] and after off[S] stay as they were."""
    sizes = [100, 20000, 0, 3, 9000]
    start = 777
    off = offsets_of(sizes, start)
    n = int(off[-1]) + 555
    announce(f"batched offset start n={n}")
    k = inputs.uniform_keys(n, 71)
    v = inputs.index_values(n)
    gk, gv = run_batched(k, v, off)
    wk, wv = oracle.lsd_sort_segmented(k, v, off)
    check((gk, gv), (wk, wv), "offset start")
    assert np.array_equal(gk[:start], k[:start]) and np.array_equal(gk[int(off[-1]):], k[int(off[-1]):])


def test_one_segment_matches_single_sort():
    n = (1 << 20) + 3
    announce(f"batched one segment n={n}")
    k = inputs.uniform_keys(n, 72)
    v = inputs.index_values(n)
    off = np.array([0, n], dtype=np.uint32)
    check(run_batched(k, v, off), oracle.lsd_sort(k, v), "one segment")


def test_many_tiny_segments():
    rng = np.random.default_rng(73)
    sizes = rng.integers(0, 6, size=100_000)
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched tiny segments S={len(sizes)} n={n}")
    k = rng.integers(0, 4, size=n, dtype=np.uint32) * np.uint32(0x01010101)
    v = inputs.index_values(n)
    check(run_batched(k, v, off), oracle.lsd_sort_segmented(k, v, off), "tiny")


def test_empty_calls():
    import torch
    announce("batched empty calls")
    k = torch.zeros(4, dtype=torch.int32, device="cuda")
    rts.sort_pairs_batched(k, None, torch.zeros(1, dtype=torch.int32, device="cuda"), 0)
    rts.sort_pairs_batched(k, None, torch.tensor([0, 0, 0], dtype=torch.int32, device="cuda"), 0)
    sync()


def test_validate_reports_malformed_offsets():
    """A segment reaching past max_total is left unsorted and reported; the
    well-formed segment before it is sorted."""
    n = 6000
    k = inputs.uniform_keys(n, 74)
    v = inputs.index_values(n)
    off = np.array([0, 1000, 6000], dtype=np.uint32)
    announce("batched validate past max_total")
    kd, vd, od = to_dev(k), to_dev(v), to_dev(off)
    with pytest.raises(RtError) as e:
        rts.sort_batched_ex(kd, vd, od, 2000, validate=True)
    assert e.value.status == RT_ERR_INVALID_ARG
    gk, gv = to_host(kd), to_host(vd)
    wk, wv = oracle.lsd_sort(k[:1000], v[:1000])
    assert np.array_equal(gk[:1000], wk) and np.array_equal(gv[:1000], wv)
    assert np.array_equal(gk[1000:], k[1000:]) and np.array_equal(gv[1000:], v[1000:])
    announce("batched validate decreasing offsets")
    off2 = np.array([0, 3000, 2000], dtype=np.uint32)
    kd, vd = to_dev(k), to_dev(v)
    with pytest.raises(RtError):
        rts.sort_batched_ex(kd, vd, to_dev(off2), n, validate=True)
    gk = to_host(kd)
    assert np.array_equal(gk[:3000], oracle.lsd_sort(k[:3000])[0])
    # and a well-formed call through the same path reports nothing
    kd, vd = to_dev(k), to_dev(v)
    rts.sort_batched_ex(kd, vd, to_dev(off), n, validate=True)
    check((to_host(kd), to_host(vd)), oracle.lsd_sort_segmented(k, v, off), "validated")


def test_graph_capture_replays():
    """With a caller workspace the call only enqueues kernels: captured once
    into a graph, every replay sorts its fresh input like the eager call."""
    import torch
    sizes = [5000, 30000, 100, 17000, 2]
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched graph capture n={n}")
    k_h = inputs.uniform_keys(n, 75)
    v_h = inputs.index_values(n)
    want = oracle.lsd_sort_segmented(k_h, v_h, off)
    k0, v0, o = to_dev(k_h), to_dev(v_h), to_dev(off)
    k, v = k0.clone(), v0.clone()
    ws = torch.empty(rts.batched_workspace_bytes(len(sizes), n, True), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rts.sort_batched_ex(k, v, o, n, workspace=ws, stream=s)  # eager warm-up
    torch.cuda.current_stream().wait_stream(s)
    sync()
    check((to_host(k), to_host(v)), want, "eager")
    g = torch.cuda.CUDAGraph()
    k.copy_(k0)
    v.copy_(v0)
    sync()
    with torch.cuda.graph(g, stream=s):
        rts.sort_batched_ex(k, v, o, n, workspace=ws, stream=s)
    for rep in range(3):
        k.copy_(k0)
        v.copy_(v0)
        sync()
        g.replay()
        sync()
        check((to_host(k), to_host(v)), want, f"replay {rep}")
        # eager work between replays
        k2, v2 = k0.clone(), v0.clone()
        rts.sort_pairs_batched(k2, v2, o, n)
        sync()
        check((to_host(k2), to_host(v2)), want, f"eager after replay {rep}")
