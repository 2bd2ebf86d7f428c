"""The segmented sort under tuned size classes: tables other than the
built-in one (four classes of different kernel shapes; a single small class
that leaves mid-size segments to the tiled path; classes with 11-bit
digits; the 8K-item tile for the tiled passes) give the oracle's result,
bit-exact, in batched calls, the MSD-first sort and the server."""
import json

import numpy as np
import pytest

import oracle
import paper_1008_2849_amd as rts
from paper_1008_2849_amd import _lib, inputs
from paper_1008_2849_amd.api import gen_params_to_c
from paper_1008_2849_amd.server import Server
from gpu_util import announce, sync, to_dev, to_host
from test_gpu_batched import check, offsets_of, run_batched

pytestmark = pytest.mark.gpu

# (max_n, block, ipt) per class, digit bits per class, tile of the tiled passes
TABLES = {
    "four": ([(1024, 256, 4), (4096, 512, 8), (8192, 1024, 8), (16384, 1024, 16)], [8] * 4, (1024, 16)),
    "one_small": ([(2048, 256, 8)], [8], (1024, 16)),
    "wide_first": ([(4096, 256, 16), (16384, 1024, 16)], [8, 8], (1024, 16)),
    "one_wave": ([(256, 64, 4), (512, 64, 8), (1024, 128, 8), (16384, 1024, 16)], [8] * 4, (1024, 16)),
    "eleven_bits": ([(256, 64, 4), (1024, 256, 4), (4096, 256, 16), (8192, 512, 16)], [11, 11, 11, 11],
                    (1024, 16)),
    "mixed_tile8k": ([(512, 64, 8), (2048, 256, 8), (8192, 512, 16)], [11, 8, 11], (512, 16)),
    # the sub-bucket classes of two-level MSD-first sorts of 2^28 and 2^26 items
    "tight_4k": ([(4352, 256, 17), (8192, 512, 16), (16384, 1024, 16)], [8] * 3, (1024, 16)),
    "tight_1k": ([(1152, 128, 9), (2304, 256, 9), (4352, 256, 17), (16384, 1024, 16)], [8] * 4, (1024, 16)),
}
BITS = {8: [8, 8, 8, 8], 11: [11, 11, 10]}


@pytest.fixture(params=sorted(TABLES) + ["builtin", "committed"])
def classes(request, tmp_path):
    if request.param == "builtin":
        rts.load_tuning(None)
    elif request.param == "committed":  # the autotuner's table for gfx950
        rts.load_tuning(_lib.TUNING_PATH)
    else:
        cls, bits, tile = TABLES[request.param]
        path = tmp_path / "classes.json"
        path.write_text(json.dumps({"entries": [
            {"op": "segments", "min_n": 0, "max_n": m, "digit_bits": BITS[w], "block": b, "ipt": i}
            for (m, b, i), w in zip(cls, bits)] + [
            {"op": "segments_tiled", "min_n": 0, "max_n": 0, "digit_bits": BITS[8], "block": tile[0],
             "ipt": tile[1]}]}))
        rts.load_tuning(str(path))
        assert rts.segment_classes() == cls and rts.segment_config() == (bits, tile)
    yield request.param, rts.segment_classes()
    rts.load_default_tuning()


def _edge_sizes(table):
    sizes = [0, 1, 2, 64, 100_003]
    for m, _, _ in table:
        sizes += [m - 1, m, m + 1]
    return sizes


def test_batched(classes):
    name, table = classes
    rng = np.random.default_rng(len(name))
    sizes = _edge_sizes(table) * 2
    rng.shuffle(sizes)
    off = offsets_of(sizes)
    n = int(off[-1])
    announce(f"batched under classes {name}, {len(sizes)} segments n={n}")
    k = inputs.uniform_keys(n, 90 + len(name))
    v = inputs.index_values(n)
    check(run_batched(k, v, off, validate=True), oracle.lsd_sort_segmented(k, v, off), name)
    check(run_batched(k, None, off), oracle.lsd_sort_segmented(k, None, off), name + " keys")


@pytest.mark.parametrize("n", [(1 << 19) + 77, (1 << 23) + 5])
def test_msd_first(classes, n):
    """2^19 items: MSD buckets of about 2048 items, on both sides of the
    limits; 2^23: buckets of about 32K items, sorted by the tiled passes."""
    name, table = classes
    announce(f"MSD-first under classes {name} n={n}")
    k = inputs.uniform_keys(n, 95)
    v = inputs.index_values(n)
    kd, vd = to_dev(k), to_dev(v)
    rts.sort_msd_first(kd, vd, validate=True)
    sync()
    wk, wv = oracle.reverse_sort(k, v)
    assert np.array_equal(to_host(kd), wk) and np.array_equal(to_host(vd), wv)


def test_server(classes):
    import torch
    name, table = classes
    sizes = _edge_sizes(table)
    announce(f"server under classes {name}, {len(sizes)} requests")
    with Server(hbm_budget_bytes=32 << 20, max_active=32) as srv:
        pending = []
        for rid, n in enumerate(sizes):
            p = inputs.counter_params(rid % 3, inputs.SEED_SERVING, 500 + rid)
            pending.append((srv.submit_generated(gen_params_to_c(p), n), p, n))
        for t, p, n in pending:
            srv.wait(t)
            k = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            v = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            srv.fetch(t, k, v)
            sync()
            keys = inputs.counter_keys(p, n)
            wk, wv = oracle.lsd_sort(keys, np.arange(n, dtype=np.uint32))
            assert np.array_equal(to_host(k)[:n], wk) and np.array_equal(to_host(v)[:n], wv), (name, n)
