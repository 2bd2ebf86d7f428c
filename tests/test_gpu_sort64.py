"""Parity of the 64-bit-key sort with the oracle's 64-bit LSD sort,
bit-exact, on seeded inputs.

Sizes span one to many 8K-item tiles with ragged tails; the distributions
leave 0, 1, 2, 3 or all 8 passes executed (constant digits are skipped), so
every buffer path of the plan runs; values of 0, 4 and 8 bytes; every digit
decomposition and tile shape built for 64-bit keys.  Values are original
indices (8-byte values carry the index and its complement), so any
instability or lost item shows up as a value mismatch.
"""
import numpy as np
import pytest

import oracle
import paper_1008_2849_amd as rts
from paper_1008_2849_amd import inputs
from paper_1008_2849_amd.api import Config, FLAG_CHUNKS, FLAG_NO_SKIP, FLAG_ONE_CHAIN
from gpu_util import announce, sync

pytestmark = pytest.mark.gpu

TILE = 8192
SIZES = [0, 1, 2, 3, 63, 64, 65, 1000, TILE - 1, TILE, TILE + 1, 3 * TILE + 77, 100_003,
         (1 << 20) - 1, (1 << 20) + 1]


def dev64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


def dev32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32).copy()).cuda()


def host64(t):
    return t.cpu().numpy().view(np.uint64)


def host32(t):
    return t.cpu().numpy().view(np.uint32)


def values(n, vb):
    if vb == 0:
        return None
    v = inputs.index_values(n)
    return v if vb == 4 else np.stack([v, ~v], axis=1).astype(np.uint32)


def gpu_sort64(keys, vals=None, cfg=None, workspace=None):
    k = dev64(keys)
    v = None
    if vals is not None:
        v = dev32(vals) if vals.ndim == 1 else dev64(vals.view(np.uint64).reshape(-1))
    rts.sort64_ex(k, v, cfg, workspace)
    sync()
    out_v = None
    if v is not None:
        out_v = host32(v) if vals.ndim == 1 else host64(v).view(np.uint32).reshape(-1, 2)
    return host64(k), out_v


def check(got, want, what):
    gk, gv = got
    wk, wv = want
    if not np.array_equal(gk, wk):
        bad = np.nonzero(gk != wk)[0]
        raise AssertionError(f"{what}: keys differ at {bad.size} positions, first {bad[:5]}")
    if wv is not None and not np.array_equal(gv, wv):
        bad = np.nonzero((gv != wv).reshape(gv.shape[0], -1).any(axis=1))[0]
        raise AssertionError(f"{what}: values differ at {bad.size} positions, first {bad[:5]}")


@pytest.mark.parametrize("vb", [0, 4, 8])
@pytest.mark.parametrize("n", SIZES)
def test_uniform_sizes(n, vb):
    announce(f"64-bit keys uniform n={n} value_bytes={vb}")
    k = inputs.keys64("uniform", n, 700 + n % 997)
    v = values(n, vb)
    check(gpu_sort64(k, v), oracle.lsd_sort64(k, v), f"n={n} vb={vb}")


def _dists(n):
    idx = np.arange(n, dtype=np.uint64)
    u = inputs.keys64("uniform", n, 710)
    return {
        "small": inputs.keys64("small", n, 711),          # 3 executed passes
        "high": inputs.keys64("high", n, 712),            # 2 executed passes
        "low32": inputs.keys64("low32", n, 713),          # 4 executed passes
        "and2": inputs.keys64("and2", n, 714),
        "one_byte": (u & np.uint64(0xFF)) << np.uint64(32),  # 1 executed pass: copied back
        "all_equal": np.full(n, 0xFEDCBA9876543210, dtype=np.uint64),  # nothing executed
        "sorted": idx,
        "reversed": idx[::-1].copy(),
        "two_values": np.where(u & np.uint64(1), np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0)),
        "dict16": u[:16][inputs.uniform_keys(n, 715) % 16],
    }


@pytest.mark.parametrize("dist", list(_dists(16).keys()))
def test_distributions(dist):
    n = (1 << 20) + 123
    announce(f"64-bit keys dist={dist} n={n}")
    k = _dists(n)[dist]
    v = values(n, 4)
    check(gpu_sort64(k, v), oracle.lsd_sort64(k, v), dist)
    check(gpu_sort64(k), oracle.lsd_sort64(k), dist + " keys only")


@pytest.mark.parametrize("dist", list(_dists(16).keys()))
def test_chunk_flags(dist):
    """XCD chunks forced at a size below the default's threshold (8 chunks of
    uneven tile counts, chunk ends inside tiles), and one chain, both give
    the oracle's result, with 4- and 8-byte values."""
    n = 23 * TILE + 4097
    announce(f"64-bit keys chunk flags dist={dist} n={n}")
    k = _dists(n)[dist]
    want4 = oracle.lsd_sort64(k, values(n, 4))
    for flags in (FLAG_CHUNKS, FLAG_CHUNKS | FLAG_NO_SKIP, FLAG_ONE_CHAIN):
        cfg = Config((8,) * 8, 1024, 8, flags)
        check(gpu_sort64(k, values(n, 4), cfg), want4, f"{dist} flags={flags}")
    cfg = Config((8,) * 8, 512, 16, FLAG_CHUNKS)
    v8 = values(n, 8)
    check(gpu_sort64(k, v8, cfg), oracle.lsd_sort64(k, v8), f"{dist} 8-byte values")


@pytest.mark.parametrize("dist,expected", [("uniform", 1), ("and2", 0), ("dict16", 0)])
def test_probed_size(dist, expected):
    """At 2^25 items the default samples the keys and picks chunks (uniform)
    or one chain (skewed: digit 0 in 10 % of AND-2 keys, a 16-key
    dictionary): the decision is the expected one, and the result is the
    oracle's either way."""
    n = (1 << 25) + 33
    announce(f"64-bit keys probed dist={dist} n={n}")
    k = inputs.keys64("uniform", n, 740) if dist == "uniform" else _dists(n)[dist]
    v = values(n, 4)
    assert rts.chunk_decision(dev64(k), value_bytes=4) == expected, dist
    check(gpu_sort64(k, v), oracle.lsd_sort64(k, v), dist)


CONFIGS = [((8,) * 8, 1024, 8), ((8,) * 8, 512, 16), ((11, 11, 11, 11, 10, 10), 512, 8),
           ((10, 9, 9, 9, 9, 9, 9), 512, 8), ((8, 8, 8, 8, 8, 8, 8, 8), 1024, 8),
           ((8,) * 8, 1024, 16), ((8,) * 8, 1024, 12)]


@pytest.mark.parametrize("flags", [0, FLAG_NO_SKIP])
@pytest.mark.parametrize("ci", range(len(CONFIGS)))
def test_configs(ci, flags):
    widths, block, ipt = CONFIGS[ci]
    n = 5 * (block * ipt) + 1234
    announce(f"64-bit keys config {widths} {block}x{ipt} flags={flags} n={n}")
    cfg = Config(widths, block, ipt, flags)
    for dist, k in [("uniform", inputs.keys64("uniform", n, 720 + ci)), ("small", inputs.keys64("small", n, 730))]:
        for vb in (0, 4, 8):
            v = values(n, vb)
            check(gpu_sort64(k, v, cfg), oracle.lsd_sort64(k, v, widths), f"{dist} {widths} vb={vb}")


def test_explicit_workspace_and_repeat():
    import torch
    n = 200_001
    announce(f"64-bit keys explicit workspace n={n}")
    k = inputs.keys64("and2", n, 740)
    v = values(n, 8)
    want = oracle.lsd_sort64(k, v)
    ws = torch.empty(rts.workspace_bytes64(n, 8), dtype=torch.uint8, device="cuda")
    for rep in range(3):
        check(gpu_sort64(k, v, None, ws), want, f"rep {rep}")


def test_full_size_workload_properties():
    """2^28 uniform 64-bit keys with index values (the measured 64-bit
    workload): the output is checked by the properties that fix a stable sort
    of original indices, and a sample of output positions against the
    oracle's sort of the keys alone."""
    import torch
    w = inputs.WORKLOADS["pairs64_256m_uniform"]
    n = w.n
    announce(f"64-bit keys full workload n={n}")
    k_h, _ = inputs.make_workload(w)
    k = dev64(k_h)
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    rts.sort_pairs64(k, v)
    sync()
    gk, gv = host64(k), host32(v)
    del k, v
    torch.cuda.empty_cache()
    assert np.all(np.bincount(gv, minlength=n) == 1)
    assert np.array_equal(k_h[gv], gk)
    assert np.all(gk[1:] >= gk[:-1])
    eq = gk[1:] == gk[:-1]
    assert np.all(gv[1:][eq] > gv[:-1][eq])
    # sampled: the sorted keys at every 4099th position equal the oracle's
    ok, _ = oracle.lsd_sort64(k_h, None)
    idx = np.arange(0, n, 4099)
    assert np.array_equal(gk[idx], ok[idx])
