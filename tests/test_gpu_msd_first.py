"""Parity of the MSD-first ("reverse sorting") path with the oracle's
Algorithm 2 definition, bit-exact, on seeded inputs.

The MSD buckets become segments of the segmented sort, so the cases aim at
its edges: buckets of 0 and 1 items, buckets at and just past each
whole-in-LDS class limit (2048, 8192, 16384) and the tile size, every item in
one bucket (constant top byte), two extreme buckets, and the full 2^28-pair
workload in the configuration the benchmark times.  Each runs with one MSD
level and with two; with two, the sub-buckets (top 16 bits) get the same
edge cases.
"""
import numpy as np
import pytest

import oracle
import paper_1008_2849_amd as rts
from paper_1008_2849_amd import inputs
from gpu_util import announce, sync, to_dev, to_host
from test_gpu_sort import SIZES, _dist_cases, assert_same

pytestmark = pytest.mark.gpu


def gpu_msd_first(keys, vals=None, **kw):
    k = to_dev(keys)
    v = None if vals is None else to_dev(vals)
    rts.sort_msd_first(k, v, **kw)
    sync()
    return to_host(k), (None if v is None else to_host(v))


LEVELS = [1, 2]


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("n", SIZES)
def test_pairs_uniform_sizes(n, levels):
    announce(f"msd-first pairs uniform n={n} levels={levels}")
    k = inputs.uniform_keys(n, 300 + n % 997)
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True, levels=levels), oracle.reverse_sort(k, v), f"n={n}")


@pytest.mark.parametrize("levels", [None] + LEVELS)
@pytest.mark.parametrize("n", [2, 65, 16385, (1 << 20) + 1])
def test_keys_uniform_sizes(n, levels):
    announce(f"msd-first keys uniform n={n} levels={levels}")
    k = inputs.uniform_keys(n, 400 + n % 991)
    assert_same(gpu_msd_first(k, levels=levels), oracle.reverse_sort(k), f"n={n}")


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("dist", list(_dist_cases(8).keys()))
def test_distributions_pairs(dist, levels):
    n = (1 << 20) + 123
    announce(f"msd-first pairs dist={dist} n={n} levels={levels}")
    k = _dist_cases(n)[dist]
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True, levels=levels), oracle.reverse_sort(k, v), dist)


def _bucketed_keys(counts, seed):
    """Keys whose MSD bucket d holds counts[d] items, lower 24 bits uniform,
    in a shuffled order."""
    rng = np.random.default_rng(seed)
    msd = np.repeat(np.arange(len(counts), dtype=np.uint32), counts)
    low = rng.integers(0, 1 << 24, size=msd.size, dtype=np.uint32)
    k = (msd << np.uint32(24)) | low
    rng.shuffle(k)
    return k


@pytest.mark.parametrize("levels", LEVELS)
@pytest.mark.parametrize("case", ["class_edges", "tile_edges", "sparse", "one_heavy"])
def test_bucket_size_edges(case, levels):
    counts = np.zeros(256, dtype=np.int64)
    if case == "class_edges":
        for d, c in zip(range(0, 256, 16), [0, 1, 2, 2047, 2048, 2049, 8191, 8192, 8193, 16383, 16384,
                                             16385, 3, 64, 65, 100]):
            counts[d] = c
    elif case == "tile_edges":
        for d, c in zip([1, 7, 99, 200, 255], [16384 * 2, 16384 * 2 + 1, 16384 * 5 - 1, 16385, 16384 * 3]):
            counts[d] = c
    elif case == "sparse":
        counts[[0, 255]] = [70_001, 1]
    else:
        counts[:] = 3
        counts[128] = 400_000
    n = int(counts.sum())
    announce(f"msd-first bucket sizes {case} n={n} levels={levels}")
    k = _bucketed_keys(counts, 500 + len(case))
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True, levels=levels), oracle.reverse_sort(k, v), case)
    assert_same(gpu_msd_first(k, levels=levels), oracle.reverse_sort(k), case + " keys")


def _subbucketed_keys(counts, seed):
    """Keys whose sub-bucket s (top 16 bits) holds counts[s] items, lower 16
    bits uniform, in a shuffled order."""
    rng = np.random.default_rng(seed)
    top = np.repeat(np.arange(len(counts), dtype=np.uint32), counts)
    low = rng.integers(0, 1 << 16, size=top.size, dtype=np.uint32)
    k = (top << np.uint32(16)) | low
    rng.shuffle(k)
    return k


@pytest.mark.parametrize("case", ["class_edges", "tile_edges", "one_bucket", "tiny_buckets"])
def test_sub_bucket_size_edges(case):
    """Two MSD levels: sub-buckets of 0 and 1 items, at and just past each
    whole-in-LDS class limit and the tile size (two tiled passes), all of a
    bucket's items in one sub-bucket, and buckets of one item (no digit-2
    counts) beside full ones."""
    counts = np.zeros(1 << 16, dtype=np.int64)
    if case == "class_edges":
        for i, c in enumerate([0, 1, 2, 3, 64, 65, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097,
                               8191, 8192, 8193, 16383, 16384, 16385]):
            counts[(i * 7919) % (1 << 16)] = c
    elif case == "tile_edges":
        for s, c in zip([5, 300, 301, 40000, 65535], [16384 * 2, 16384 * 2 + 1, 16384 * 5 - 1, 16385, 16384 * 3]):
            counts[s] = c
    elif case == "one_bucket":
        counts[(77 << 8) + 3] = 300_000  # every item of bucket 77 in one sub-bucket
        counts[(78 << 8):(79 << 8)] = 5
    else:
        counts[0::256] = 1  # buckets of one item
        counts[(200 << 8):(201 << 8)] = 700  # and one full bucket
        counts[65535] = 2
    n = int(counts.sum())
    announce(f"msd-first sub-bucket sizes {case} n={n}")
    k = _subbucketed_keys(counts, 700 + len(case))
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True, levels=2), oracle.reverse_sort(k, v), case)
    assert_same(gpu_msd_first(k, levels=2), oracle.reverse_sort(k), case + " keys")


@pytest.mark.parametrize("n", [(1 << 26) + 12345, (1 << 27) + 777])
def test_two_levels_sized_classes(n):
    """Sizes whose sub-buckets (about 1024 and 2048 items) take the classes
    sized to them, by default: the whole output against the oracle."""
    announce(f"msd-first default two levels n={n}")
    k = inputs.uniform_keys(n, 800 + n % 97)
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True), oracle.reverse_sort(k, v), f"n={n}")


@pytest.mark.parametrize("dist", ["and4", "zipf16", "top_00", "low_byte_only", "sorted"])
def test_two_levels_skewed_at_size(dist):
    """Two levels by default (2^26 + 99 items) on skewed keys: sub-buckets
    far from the uniform mean, the largest through the persistent tiled
    passes, the smallest empty; pairs and keys only, against the oracle."""
    n = (1 << 26) + 99
    announce(f"msd-first default two levels dist={dist} n={n}")
    k = _dist_cases(n)[dist]
    v = inputs.index_values(n)
    assert_same(gpu_msd_first(k, v, validate=True), oracle.reverse_sort(k, v), dist)
    assert_same(gpu_msd_first(k), oracle.reverse_sort(k), dist + " keys")


@pytest.mark.parametrize("levels", LEVELS)
def test_explicit_workspace_repeat_and_graph(levels):
    """A caller workspace; three eager calls and a captured graph replayed
    three times (with eager work between) all give the oracle's result."""
    import torch
    n = 3 * 16384 + 4321
    announce(f"msd-first workspace + graph n={n} levels={levels}")
    k_h = inputs.uniform_keys(n, 600)
    v_h = inputs.index_values(n)
    want = oracle.reverse_sort(k_h, v_h)
    ws = torch.empty(rts.msd_first_workspace_bytes(n, True), dtype=torch.uint8, device="cuda")
    k0, v0 = to_dev(k_h), to_dev(v_h)
    k, v = k0.clone(), v0.clone()
    for rep in range(3):
        k.copy_(k0)
        v.copy_(v0)
        rts.sort_msd_first(k, v, workspace=ws, levels=levels)
        sync()
        assert_same((to_host(k), to_host(v)), want, f"eager {rep}")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        k.copy_(k0)
        v.copy_(v0)
        rts.sort_msd_first(k, v, workspace=ws, stream=s, levels=levels)  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        rts.sort_msd_first(k, v, workspace=ws, stream=s, levels=levels)
    for rep in range(3):
        k.copy_(k0)
        v.copy_(v0)
        sync()
        g.replay()
        sync()
        assert_same((to_host(k), to_host(v)), want, f"replay {rep}")
        k2, v2 = k0.clone(), v0.clone()
        rts.sort_msd_first(k2, v2, levels=levels)
        sync()
        assert_same((to_host(k2), to_host(v2)), want, f"eager after replay {rep}")


def test_headline_workload_full_size_sampled():
    """2^28 uniform pairs, as the benchmark runs it.  The oracle sorts a
    sample of MSD buckets (each is the stable sort of the items with that top
    byte, in input order); the whole output is checked by the properties that
    fix a stable sort of original indices."""
    import torch
    w = inputs.WORKLOADS["pairs_256m_uniform"]
    n = w.n
    announce(f"msd-first full workload n={n}")
    k_h, _ = inputs.make_workload(w)
    k = to_dev(k_h)
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    rts.sort_msd_first(k, v, validate=True)
    sync()
    gk, gv = to_host(k), to_host(v)
    del k, v
    torch.cuda.empty_cache()
    msd = (k_h >> np.uint32(24)).astype(np.int64)
    counts = np.bincount(msd, minlength=256)
    starts = np.concatenate([[0], np.cumsum(counts)])
    for d in [0, 1, 77, 128, 254, 255]:
        idx = np.nonzero(msd == d)[0].astype(np.uint32)
        wk, wv = oracle.reverse_sort(k_h[idx], idx)
        a, b = int(starts[d]), int(starts[d + 1])
        assert np.array_equal(gk[a:b], wk) and np.array_equal(gv[a:b], wv), f"bucket {d}"
    assert np.all(np.bincount(gv, minlength=n) == 1)
    assert np.array_equal(k_h[gv], gk)
    assert np.all(gk[1:] >= gk[:-1])
    eq = gk[1:] == gk[:-1]
    assert np.all(gv[1:][eq] > gv[:-1][eq])


@pytest.mark.parametrize("levels", LEVELS)
def test_full_size_keys_only(levels):
    """2^28 uniform keys without values, each form: the output equals numpy's
    sort of the input (for keys alone a stable sort and any sort agree), and
    a sample of MSD buckets equals the oracle's sort of that bucket."""
    import torch
    n = 1 << 28
    announce(f"msd-first full size keys only levels={levels}")
    k_h = inputs.uniform_keys(n, 21)
    k = to_dev(k_h)
    rts.sort_msd_first(k, validate=True, levels=levels)
    sync()
    gk = to_host(k)
    del k
    torch.cuda.empty_cache()
    assert np.array_equal(gk, np.sort(k_h))
    msd = (k_h >> np.uint32(24)).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(np.bincount(msd, minlength=256))])
    for d in [3, 200]:
        wk, _ = oracle.reverse_sort(k_h[msd == d])
        assert np.array_equal(gk[int(starts[d]):int(starts[d + 1])], wk), f"bucket {d}"
