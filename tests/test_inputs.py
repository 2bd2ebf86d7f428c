"""The seeded input generators draw what their workload descriptions say."""
import os

import numpy as np
import pytest

from paper_1008_2849_amd import inputs


def test_seeded_and_deterministic():
    a = inputs.uniform_keys(1 << 12, 1)
    b = inputs.uniform_keys(1 << 12, 1)
    c = inputs.uniform_keys(1 << 12, 2)
    assert a.dtype == np.uint32 and np.array_equal(a, b) and not np.array_equal(a, c)


@pytest.mark.parametrize("k", [2, 4, 8])
def test_and_of_k_bit_frequency(k):
    n = 1 << 18
    keys = inputs.and_keys(n, k, inputs.SEED_AND[k])
    bits = np.unpackbits(keys.view(np.uint8)).reshape(n, 32).mean(axis=0)
    p = 2.0 ** -k
    sd = np.sqrt(p * (1 - p) / n)
    assert np.all(np.abs(bits - p) < 6 * sd)


def test_top_byte_constant():
    keys = inputs.top_byte_keys(1 << 16, 0xA5, 34)
    assert np.all((keys >> 24) == 0xA5)
    assert len(np.unique(keys & 0xFFFFFF)) > (1 << 16) * 0.99


def test_zipf16_frequencies():
    n = 1 << 18
    keys = inputs.zipf16_keys(n, 35)
    d = inputs.zipf16_dictionary(35)
    assert len(set(d.tolist())) == 16
    counts = np.array([(keys == x).sum() for x in d])
    assert counts.sum() == n
    p = inputs.zipf_probabilities(16, 1.2)
    assert abs(p[0] - 0.3653) < 1e-3 and abs(p[15] - 0.0131) < 1e-3
    chi2 = (((counts - n * p) ** 2) / (n * p)).sum()
    assert chi2 < 50.0  # 15 degrees of freedom; p ~ 1e-5 at 50


def test_batched_sizes():
    sizes = inputs.batched_sizes()
    assert sizes.size == 4096
    assert int(sizes.sum()) <= 2**27
    assert sizes.min() >= 64
    off = inputs.segment_offsets(sizes)
    assert off[0] == 0 and off[-1] == sizes.sum() and np.all(np.diff(off.astype(np.int64)) >= 0)
    # uncapped draws keep the log-uniform shape
    raw = inputs.batched_sizes(num_segments=4096, cap=2**40)
    lg = np.log2(raw.astype(np.float64))
    assert 6.0 <= lg.min() and lg.max() < 20.0
    assert abs(lg.mean() - 13.0) < 0.3


def test_poisson_arrivals():
    t = inputs.poisson_arrivals(1000.0, 20000, 5)
    gaps = np.diff(t)
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() - 1e-3) < 5e-5


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 seeded with 1234567 (reference vector of
    # the published generator).
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [int(x) for x in inputs.splitmix64_words(1234567, 0, 5)] == want


def test_counter_keys_distributions():
    n = 1 << 16
    pu = inputs.counter_params(inputs.DIST_UNIFORM, 5, 0)
    ku = inputs.counter_keys(pu, n)
    assert len(np.unique(ku)) > n * 0.99
    # any window re-generated from its first index is the same data
    assert np.array_equal(inputs.counter_keys(pu, 100, first=1000), ku[1000:1100])
    pa = inputs.counter_params(inputs.DIST_AND4, 5, 1)
    ka = inputs.counter_keys(pa, n)
    bits = np.unpackbits(ka.view(np.uint8)).mean()
    assert abs(bits - 1 / 16) < 0.005
    assert np.array_equal(inputs.counter_keys(pa, 64, first=4096), ka[4096:4160])
    pz = inputs.counter_params(inputs.DIST_ZIPF16, 5, 2)
    kz = inputs.counter_keys(pz, n)
    assert set(np.unique(kz).tolist()) <= set(pz.dictionary)
    top = (kz == pz.dictionary[0]).mean()
    assert abs(top - 0.3653) < 0.01
    t = inputs.zipf16_thresholds()
    assert t[-1] == 2**32 and np.all(np.diff(t.astype(np.int64)) > 0)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
