"""Sorts past 2^30 items, where the lookback words become 64-bit and element
offsets no longer fit 32-bit byte offsets: the single-array sort (8-bit and
11/11/10-bit digits), the MSD-first sort (whose segmented passes switch
too) and 64-bit keys, with and without values.

At this size the oracle is checked on the output's defining properties, on
the device: keys ascend (unsigned), the values are a permutation of the
original indices, every key arrives with its own index, and equal keys keep
index order -- together they fix the stable sort uniquely.  Inputs come from
the library's counter-based generator (checked against its host definition
in test_gpu_sort.py) or torch's seeded device generator.
"""
import pytest

import paper_1008_2849_amd as rts
from paper_1008_2849_amd import inputs
from gpu_util import announce, sync

pytestmark = pytest.mark.gpu

N = (1 << 30) + 4321


def _check_pairs(k0, k, v):
    import torch
    ku = k.to(torch.int64) & 0xFFFFFFFF
    assert bool((ku[1:] >= ku[:-1]).all()), "keys ascend"
    vl = v.to(torch.int64)
    assert bool(((vl >= 0) & (vl < k.numel())).all()), "values in range"
    assert bool((torch.bincount(vl, minlength=k.numel()) == 1).all()), "values are a permutation"
    assert bool(torch.equal(k0[vl], k)), "each key arrives with its own index"
    eq = ku[1:] == ku[:-1]
    assert bool((vl[1:][eq] > vl[:-1][eq]).all()), "equal keys keep index order"


@pytest.mark.parametrize("path", ["lsd", "msd_first"])
def test_pairs_past_2_30(path):
    import torch
    announce(f"{path} pairs n={N}")
    k = torch.empty(N, dtype=torch.int32, device="cuda")
    v = torch.empty(N, dtype=torch.int32, device="cuda")
    rts.generate(k, v, inputs.counter_params(inputs.DIST_AND4, 61, 0))  # low-entropy keys, values = index
    k0 = k.clone()
    if path == "lsd":
        rts.sort_pairs(k, v)
    else:
        rts.sort_msd_first(k, v, validate=True)
    sync()
    _check_pairs(k0, k, v)
    del k, v, k0
    torch.cuda.empty_cache()


def test_eleven_bit_digits_past_2_30():
    """11/11/10-bit digits (three passes, 2048-word lookback rows) past 2^30
    items, where those rows' words are 64-bit: the properties of the stable
    sort, and no lookback gave up (RT_FLAG_VALIDATE)."""
    import torch
    from paper_1008_2849_amd.api import Config, FLAG_VALIDATE
    announce(f"11/11/10 pairs n={N}")
    k = torch.empty(N, dtype=torch.int32, device="cuda")
    v = torch.empty(N, dtype=torch.int32, device="cuda")
    rts.generate(k, v, inputs.counter_params(inputs.DIST_UNIFORM, 63, 0))
    k0 = k.clone()
    rts.sort_ex(k, v, Config((11, 11, 10), 512, 16, FLAG_VALIDATE))
    sync()
    _check_pairs(k0, k, v)
    del k, v, k0
    torch.cuda.empty_cache()


def test_pairs64_past_2_30():
    """64-bit keys with 4-byte values past 2^30 items: 16K-item tiles whose
    keys and values are staged one after the other, 64-bit lookback words,
    64-bit element offsets.  Checked by the stable sort's properties."""
    import torch
    announce(f"64-bit keys with values n={N}")
    g = torch.Generator(device="cuda")
    g.manual_seed(64)
    # few distinct high bits: long runs of equal keys exercise stability
    k = torch.randint(0, 1 << 40, (N,), dtype=torch.int64, device="cuda", generator=g) << 20
    v = torch.arange(N, dtype=torch.int32, device="cuda")
    k0 = k.clone()
    rts.sort64_ex(k, v)
    sync()
    assert bool((k[1:] >= k[:-1]).all()), "keys ascend"  # all keys below 2^60: signed order is unsigned order
    vl = v.to(torch.int64)
    assert bool((torch.bincount(vl, minlength=N) == 1).all()), "values are a permutation"
    assert bool(torch.equal(k0[vl], k)), "each key arrives with its own index"
    eq = k[1:] == k[:-1]
    assert bool((vl[1:][eq] > vl[:-1][eq]).all()), "equal keys keep index order"
    del k, v, k0, vl, eq
    torch.cuda.empty_cache()


def test_keys64_past_2_30():
    import torch
    announce(f"64-bit keys n={N}")
    g = torch.Generator(device="cuda")
    g.manual_seed(62)
    k = torch.randint(-(1 << 63), (1 << 63) - 1, (N,), dtype=torch.int64, device="cuda", generator=g)
    sign = torch.tensor(-(1 << 63), dtype=torch.int64, device="cuda")
    want = torch.sort(k ^ sign).values ^ sign  # unsigned ascending order
    rts.sort_keys64(k)
    sync()
    assert bool(torch.equal(k, want))
    del k, want
    torch.cuda.empty_cache()
