"""Pins for the CPU oracle: it is checked against things other than itself.

* hand-worked examples derived from the paper's description of counting sort
  and LSD radix sort (tests/golden/, each fixture states its passage);
* brute force on tiny inputs: the rank definition of a stable sort, in pure
  Python, exhaustively for n <= 5 over a 9-value alphabet that exercises every
  byte position and the sign bit, and on random heavy-tie inputs;
* a library routine the method reduces to: numpy's stable argsort;
* closed forms (identity, reversal, all-equal, bit-reversal permutation) and
  invariants (nondecreasing, permutation, stability, digit-width invariance,
  histogram sums).

Each pin is also run against oracle builds with a planted mistake (dropped
pass, reversed digit order, unstable scatter, wrong mask, ...), and each of
those builds must fail at least one pin.
"""
import itertools
import json
import os
import tempfile

import numpy as np
import pytest

import oracle
from paper_1008_2849_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALPHABET = [0, 1, 0xFF, 0x100, 0xFFFF, 0x10000, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]


def _hex_list(xs):
    return np.array([int(x, 16) for x in xs], dtype=np.uint32)


def _stable_reference(keys, vals):
    perm = np.argsort(keys, kind="stable")
    return keys[perm], (None if vals is None else vals[perm])


# ---------------------------------------------------------------- pins ----

def pin_worked_example(so):
    with open(os.path.join(GOLDEN, "worked_example_8x4.json")) as f:
        g = json.load(f)
    k = _hex_list(g["keys"])
    v = np.array(g["values"], dtype=np.uint32)
    for p in g["passes"]:
        hist = oracle.digit_histogram(k, p["shift"], 8, so=so)
        want = np.zeros(256, dtype=np.uint64)
        for d, c in p["histogram_nonzero"].items():
            want[int(d)] = c
        assert np.array_equal(hist, want), f"histogram at shift {p['shift']}"
        k, v = oracle.counting_pass(k, v, p["shift"], 8, so=so)
        assert np.array_equal(k, _hex_list(p["keys"])), f"keys after shift {p['shift']}"
        assert np.array_equal(v, np.array(p["values"], dtype=np.uint32))
    k0 = _hex_list(g["keys"])
    v0 = np.array(g["values"], dtype=np.uint32)
    ks, vs = oracle.lsd_sort(k0, v0, g["widths"], so=so)
    assert np.array_equal(ks, _hex_list(g["sorted_keys"]))
    assert np.array_equal(vs, np.array(g["sorted_values"], dtype=np.uint32))


def pin_unsigned_order(so):
    with open(os.path.join(GOLDEN, "unsigned_order.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        ks, vs = oracle.lsd_sort(_hex_list(c["keys"]), np.array(c["values"], dtype=np.uint32),
                                 c["widths"], so=so)
        assert np.array_equal(ks, _hex_list(c["sorted_keys"])), c
        assert np.array_equal(vs, np.array(c["sorted_values"], dtype=np.uint32)), c


def _all_tuples(max_len):
    cases = []
    for length in range(0, max_len + 1):
        for t in itertools.product(range(len(ALPHABET)), repeat=length):
            cases.append([ALPHABET[i] for i in t])
    return cases


def pin_exhaustive_tiny(so, max_len=5, widths=(8, 8, 8, 8)):
    cases = _all_tuples(max_len)
    sizes = np.array([len(c) for c in cases], dtype=np.uint32)
    off = inputs.segment_offsets(sizes)
    keys = np.array([x for c in cases for x in c], dtype=np.uint32)
    vals = inputs.index_values(keys.size)
    ks, vs = oracle.lsd_sort_segmented(keys, vals, off, widths, so=so)
    for s, c in enumerate(cases):
        lo, hi = int(off[s]), int(off[s + 1])
        bk, bv = oracle.brute_stable_sort(c, list(range(lo, hi)))
        assert list(ks[lo:hi]) == bk and list(vs[lo:hi]) == bv, (c, widths)
    # the unsegmented entry point on a slice of the same cases
    for c in cases[:: max(1, len(cases) // 400)]:
        ks1, vs1 = oracle.lsd_sort(np.array(c, dtype=np.uint32),
                                   np.arange(len(c), dtype=np.uint32), widths, so=so)
        bk, bv = oracle.brute_stable_sort(c, list(range(len(c))))
        assert list(ks1) == bk and list(vs1) == bv, c


def pin_heavy_ties(so):
    rng = np.random.default_rng(123)
    alpha = np.array([0x00000000, 0x80000001, 0x0000FF00], dtype=np.uint32)
    for _ in range(300):
        n = int(rng.integers(0, 65))
        k = alpha[rng.integers(0, 3, size=n)]
        v = np.arange(n, dtype=np.uint32)
        ks, vs = oracle.lsd_sort(k, v, so=so)
        bk, bv = oracle.brute_stable_sort(list(k), list(v))
        assert list(ks) == bk and list(vs) == bv


def pin_numpy_stable(so, n=1 << 14):
    gens = {
        "uniform": inputs.uniform_keys(n, 7),
        "and2": inputs.and_keys(n, 2, 8),
        "and8": inputs.and_keys(n, 8, 9),
        "top_a5": inputs.top_byte_keys(n, 0xA5, 10),
        "top_00": inputs.top_byte_keys(n, 0x00, 11),
        "zipf16": inputs.zipf16_keys(n, 12),
        "small_range": (inputs.uniform_keys(n, 13) % 37).astype(np.uint32),
    }
    for name, k in gens.items():
        v = inputs.index_values(n)
        for widths in [(8, 8, 8, 8), (11, 11, 10)]:
            ks, vs = oracle.lsd_sort(k, v, widths, so=so)
            rk, rv = _stable_reference(k, v)
            assert np.array_equal(ks, rk), (name, widths)
            assert np.array_equal(vs, rv), (name, widths)
        ko, none = oracle.lsd_sort(k, None, so=so)
        assert none is None and np.array_equal(ko, np.sort(k)), name


def pin_closed_forms(so, m=12):
    n = 1 << m
    idx = np.arange(n, dtype=np.uint32)
    # already sorted -> identity
    ks, vs = oracle.lsd_sort(idx, idx, so=so)
    assert np.array_equal(ks, idx) and np.array_equal(vs, idx)
    # reversed -> keys 0..n-1 with values n-1..0
    rev = idx[::-1].copy()
    ks, vs = oracle.lsd_sort(rev, idx, so=so)
    assert np.array_equal(ks, idx) and np.array_equal(vs, rev)
    # all keys equal -> identity permutation of the values
    same = np.full(n, 0xDEADBEEF, dtype=np.uint32)
    ks, vs = oracle.lsd_sort(same, idx, so=so)
    assert np.array_equal(ks, same) and np.array_equal(vs, idx)
    # bit reversal of i over m bits: sorted key j carries value bitrev(j)
    br = np.zeros(n, dtype=np.uint32)
    for b in range(m):
        br |= ((idx >> b) & 1) << (m - 1 - b)
    ks, vs = oracle.lsd_sort(br, idx, so=so)
    assert np.array_equal(ks, idx) and np.array_equal(vs, br)
    # keys spread over the high bits (only the top pass sees them)
    hi = (br.astype(np.uint64) << np.uint64(32 - m)).astype(np.uint32)
    ks, vs = oracle.lsd_sort(hi, idx, so=so)
    assert np.array_equal(vs, br)


def pin_histograms(so, n=1 << 14):
    k = inputs.uniform_keys(n, 21)
    for shift, width in [(0, 8), (8, 8), (16, 8), (24, 8), (0, 11), (11, 11), (22, 10),
                         (0, 16), (16, 16), (31, 1)]:
        h = oracle.digit_histogram(k, shift, width, so=so)
        want = np.bincount((k >> np.uint32(shift)) & np.uint32((1 << width) - 1),
                           minlength=1 << width)
        assert np.array_equal(h, want.astype(np.uint64)), (shift, width)
        assert int(h.sum()) == n


def pin_width_invariance(so, n=1 << 13):
    k = inputs.and_keys(n, 2, 31)
    v = inputs.index_values(n)
    ref = oracle.lsd_sort(k, v, (8, 8, 8, 8), so=so)
    for widths in [(11, 11, 10), (10, 11, 11), (16, 16), (4,) * 8, (1,) * 32, (5, 9, 2, 16)]:
        got = oracle.lsd_sort(k, v, widths, so=so)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), widths


def pin_invariants(so, n=1 << 15):
    for seed, k in enumerate([inputs.uniform_keys(n, 40), inputs.and_keys(n, 4, 41),
                              inputs.zipf16_keys(n, 42)]):
        v = inputs.index_values(n)
        ks, vs = oracle.lsd_sort(k, v, so=so)
        assert np.all(ks[1:] >= ks[:-1]), "nondecreasing"
        assert np.array_equal(np.sort(vs), v), "values are a permutation"
        assert np.array_equal(k[vs], ks), "each value still carries its key"
        eq = ks[1:] == ks[:-1]
        assert np.all(vs[1:][eq] > vs[:-1][eq]), "stable"
        # idempotence: sorting the output again moves nothing
        ks2, vs2 = oracle.lsd_sort(ks, np.arange(n, dtype=np.uint32), so=so)
        assert np.array_equal(ks2, ks) and np.array_equal(vs2, np.arange(n, dtype=np.uint32))


def pin_reverse_sort(so):
    """Algorithm 2's MSD-first sort against brute force, numpy and closed forms."""
    for c in _all_tuples(4):
        ks, vs = oracle.reverse_sort(np.array(c, dtype=np.uint32),
                                     np.arange(len(c), dtype=np.uint32), so=so)
        bk, bv = oracle.brute_stable_sort(c, list(range(len(c))))
        assert list(ks) == bk and list(vs) == bv, c
    rng = np.random.default_rng(321)
    alpha = np.array([0x01000000, 0x00000001, 0x01000001, 0xFF00FF00, 0x00010000], dtype=np.uint32)
    for _ in range(200):
        n = int(rng.integers(0, 65))
        k = alpha[rng.integers(0, alpha.size, size=n)]
        v = np.arange(n, dtype=np.uint32)
        ks, vs = oracle.reverse_sort(k, v, so=so)
        bk, bv = oracle.brute_stable_sort(list(k), list(v))
        assert list(ks) == bk and list(vs) == bv
    n = 1 << 14
    for name, k in {"uniform": inputs.uniform_keys(n, 70), "and2": inputs.and_keys(n, 2, 71),
                    "top_00": inputs.top_byte_keys(n, 0x00, 72), "top_a5": inputs.top_byte_keys(n, 0xA5, 73),
                    "zipf16": inputs.zipf16_keys(n, 74)}.items():
        v = inputs.index_values(n)
        ks, vs = oracle.reverse_sort(k, v, so=so)
        rk, rv = _stable_reference(k, v)
        assert np.array_equal(ks, rk) and np.array_equal(vs, rv), name
        ko, none = oracle.reverse_sort(k, None, so=so)
        assert none is None and np.array_equal(ko, rk), name
    m = 12
    idx = np.arange(1 << m, dtype=np.uint32)
    br = np.zeros(idx.size, dtype=np.uint32)
    for b in range(m):
        br |= ((idx >> b) & 1) << (m - 1 - b)
    for shift in (0, 20):  # low bits only; spread across the MSD buckets
        ks, vs = oracle.reverse_sort(br << np.uint32(shift), idx, so=so)
        assert np.array_equal(ks, idx << np.uint32(shift)) and np.array_equal(vs, br)


ALPHABET64 = [0, 1, 0xFF, 0x100, 0xFFFFFFFF, 0x100000000, 0x7FFFFFFFFFFFFFFF,
              0x8000000000000000, 0xFFFFFFFFFFFFFFFF]


def pin_sort64(so):
    """The 64-bit-key sort against brute force, numpy's stable argsort, and
    the 32-bit sort on keys below 2^32."""
    for length in range(0, 4):
        for t in itertools.product(ALPHABET64, repeat=length):
            ks, vs = oracle.lsd_sort64(np.array(t, dtype=np.uint64), np.arange(length, dtype=np.uint32), so=so)
            bk, bv = oracle.brute_stable_sort(t, list(range(length)), bits=64)
            assert [int(x) for x in ks] == bk and list(vs) == bv, t
    rng = np.random.default_rng(77)
    n = 1 << 14
    u = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    dists = {
        "uniform": u,
        "small": u >> np.uint64(44),
        "high_only": u & np.uint64(0xFFFF000000000000),
        "and2": u & rng.integers(0, 1 << 64, size=n, dtype=np.uint64),
        "dict16": rng.integers(0, 1 << 64, size=16, dtype=np.uint64)[rng.integers(0, 16, size=n)],
        "equal": np.full(n, 0x0123456789ABCDEF, dtype=np.uint64),
    }
    v1 = np.arange(n, dtype=np.uint32)
    v2 = np.stack([v1, v1 ^ np.uint32(0x5A5A5A5A)], axis=1)
    for name, k in dists.items():
        perm = np.argsort(k, kind="stable")
        for widths in [(8,) * 8, (11, 11, 11, 11, 10, 10), (16, 16, 16, 16), (5, 13, 7, 9, 16, 14)]:
            ks, vs = oracle.lsd_sort64(k, v1, widths, so=so)
            assert np.array_equal(ks, k[perm]) and np.array_equal(vs, v1[perm]), (name, widths)
        ks, vs = oracle.lsd_sort64(k, v2, so=so)
        assert np.array_equal(ks, k[perm]) and np.array_equal(vs, v2[perm]), name
        ks, none = oracle.lsd_sort64(k, None, so=so)
        assert none is None and np.array_equal(ks, np.sort(k)), name
    k32 = inputs.and_keys(n, 2, 78)
    ks, vs = oracle.lsd_sort64(k32.astype(np.uint64), v1, so=so)
    rk, rv = oracle.lsd_sort(k32, v1, so=so)
    assert np.array_equal(ks, rk.astype(np.uint64)) and np.array_equal(vs, rv)


PINS = [pin_worked_example, pin_unsigned_order, pin_closed_forms, pin_heavy_ties,
        pin_histograms, pin_numpy_stable, pin_width_invariance, pin_invariants,
        pin_exhaustive_tiny, pin_reverse_sort, pin_sort64]


# --------------------------------------------------------------- tests ----

@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(oracle.lib())


def test_exhaustive_tiny_11_11_10():
    pin_exhaustive_tiny(oracle.lib(), max_len=4, widths=(11, 11, 10))


def test_segmented_leaves_outside_untouched():
    k = inputs.uniform_keys(1000, 3)
    v = inputs.index_values(1000)
    off = np.array([100, 100, 350, 351, 900], dtype=np.uint32)
    ks, vs = oracle.lsd_sort_segmented(k, v, off)
    assert np.array_equal(ks[:100], k[:100]) and np.array_equal(ks[900:], k[900:])
    assert np.array_equal(vs[:100], v[:100]) and np.array_equal(vs[900:], v[900:])
    for lo, hi in [(100, 350), (350, 351), (351, 900)]:
        rk, rv = _stable_reference(k[lo:hi], v[lo:hi])
        assert np.array_equal(ks[lo:hi], rk) and np.array_equal(vs[lo:hi], rv)


def test_counting_pass_is_stable_partition():
    k = inputs.uniform_keys(5000, 5)
    v = inputs.index_values(5000)
    for shift, width in [(0, 8), (24, 8), (11, 11), (22, 10)]:
        d = (k >> np.uint32(shift)) & np.uint32((1 << width) - 1)
        perm = np.argsort(d, kind="stable")
        ko, vo = oracle.counting_pass(k, v, shift, width)
        assert np.array_equal(ko, k[perm]) and np.array_equal(vo, v[perm])


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.lsd_sort(np.zeros(4, np.uint32), None, (8, 8, 8))      # sums to 24
    with pytest.raises(ValueError):
        oracle.lsd_sort(np.zeros(4, np.uint32), None, (32,))          # width > 16
    with pytest.raises(ValueError):
        oracle.lsd_sort(np.zeros(4, np.uint32), None, (0, 16, 16))    # zero width
    with pytest.raises(ValueError):
        oracle.lsd_sort_segmented(np.zeros(4, np.uint32), None,
                                  np.array([0, 3, 2], np.uint32))     # decreasing
    k, v = oracle.lsd_sort(np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    assert k.size == 0 and v.size == 0


MUTANTS = {
    1: "scatter visits items in decreasing order (unstable pass)",
    2: "prefix sum over digits in descending order",
    3: "most significant pass dropped",
    4: "values not moved with their keys",
    5: "digit mask drops its top bit",
    6: "keys treated as signed",
    7: "digits taken most significant first",
    8: "MSD-first sort: every bucket written from output slot 0",
    9: "MSD-first sort: partition on digit 2",
    10: "MSD-first sort: first local pass's buckets visited in decreasing order",
    11: "64-bit keys: digit shift wraps at 32 bits",
    12: "64-bit keys: only the first of two value words moves",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=[MUTANTS[m] for m in sorted(MUTANTS)])
def test_planted_mistake_is_caught(mutant):
    with tempfile.TemporaryDirectory() as d:
        so = oracle.load(oracle.build(os.path.join(d, f"mutant{mutant}.so"), mutant=mutant))
        failed = []
        for pin in PINS:
            try:
                if pin is pin_exhaustive_tiny:
                    pin(so, max_len=3)
                else:
                    pin(so)
            except (AssertionError, ValueError):
                failed.append(pin.__name__)
        assert failed, f"no pin caught planted mistake {mutant}: {MUTANTS[mutant]}"
