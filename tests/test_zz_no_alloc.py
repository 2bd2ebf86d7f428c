"""The allocation-free sort (rt_sort_pairs_noalloc): through the C ABI it
gives rt_sort_pairs_ex's result bit for bit, on two calls in a row (the
second smaller, so the scratch holds the first call's leftovers), keys only
and pairs, and rejects a size its static scratch cannot hold before any
device work."""
import ctypes

import numpy as np
import pytest

from paper_1008_2849_amd import _lib, inputs
from gpu_util import announce, sync, to_dev, to_host

pytestmark = pytest.mark.gpu


def _ex(kd, vd, cfg_p):
    so = _lib.lib()
    st = so.rt_sort_pairs_ex(kd.data_ptr(), None if vd is None else vd.data_ptr(), kd.numel(), cfg_p,
                             None, 0, None)
    assert st == _lib.RT_OK, so.rt_last_error()


def _noalloc(kd, vd, cfg_p):
    so = _lib.lib()
    st = so.rt_sort_pairs_noalloc(kd.data_ptr(), None if vd is None else vd.data_ptr(), kd.numel(), cfg_p, None)
    assert st == _lib.RT_OK, so.rt_last_error()


@pytest.mark.parametrize("with_values", [True, False])
def test_noalloc_matches_the_workspace_sort_twice(with_values):
    import torch
    cfg = _lib.RtConfig()  # tuned defaults
    for n, seed in ((1_500_003, 121), (40_961, 122)):  # the second call is smaller
        announce(f"noalloc n={n} values={with_values}")
        keys = inputs.and_keys(n, 2, seed) if seed % 2 else inputs.uniform_keys(n, seed)
        vals = inputs.index_values(n) if with_values else None
        k1, k2 = to_dev(keys), to_dev(keys)
        v1 = to_dev(vals) if with_values else None
        v2 = to_dev(vals) if with_values else None
        _ex(k1, v1, ctypes.byref(cfg))
        _noalloc(k2, v2, ctypes.byref(cfg))
        sync()
        assert np.array_equal(to_host(k2), to_host(k1)), n
        if with_values:
            assert np.array_equal(to_host(v2), to_host(v1)), n
        assert np.all(np.diff(to_host(k2).astype(np.int64)) >= 0)


def test_noalloc_rejects_what_the_scratch_cannot_hold():
    import torch
    so = _lib.lib()
    n = 1 << 24  # 2^24 pairs need 256 MiB of temporaries
    k = torch.empty(n, dtype=torch.int32, device="cuda")
    v = torch.empty(n, dtype=torch.int32, device="cuda")
    assert so.rt_sort_pairs_noalloc(k.data_ptr(), v.data_ptr(), n, None, None) == _lib.RT_ERR_TOO_LARGE
    assert b"scratch" in so.rt_last_error()
