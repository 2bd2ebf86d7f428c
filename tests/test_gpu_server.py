"""The serving loop: every request comes back sorted exactly as the oracle
sorts it alone, whatever else shares its steps (tolerance 0: the sort is
exact).  Requests are device-generated from the counter-based generator,
which the host re-derives for the oracle, or caller-owned device arrays.
Sizes straddle the whole-in-LDS limit (16384) and the tile size; the
budget is small enough that admission has to wait for memory."""
import numpy as np
import pytest

import oracle
from paper_1008_2849_amd import inputs
from paper_1008_2849_amd.api import gen_params_to_c
from paper_1008_2849_amd.server import Server
from paper_1008_2849_amd._lib import RtError, RT_ERR_BUDGET, RT_ERR_CANCELLED, RT_ERR_INVALID_ARG, RT_ERR_NOT_FOUND
from gpu_util import announce, sync, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 100, 2048, 2049, 8192, 8193, 16384, 16385, 16384 * 2 + 5, 100_000, 300_001]


def _generated_case(srv, rid, n, dist):
    p = inputs.counter_params(dist, inputs.SEED_SERVING, rid)
    return srv.submit_generated(gen_params_to_c(p), n), p


def test_generated_mix_matches_oracle_alone():
    import torch
    rng = np.random.default_rng(5)
    sizes = list(SIZES) * 3
    rng.shuffle(sizes)
    announce(f"server generated mix of {len(sizes)} requests")
    with Server(hbm_budget_bytes=64 << 20, max_active=64) as srv:
        pending = []
        for rid, n in enumerate(sizes):
            dist = rid % 3
            t, p = _generated_case(srv, rid, n, dist)
            pending.append((t, p, n))
        for t, p, n in pending:
            lat = srv.wait(t)
            assert lat >= 0
            k = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            v = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            srv.fetch(t, k, v)
            sync()
            keys = inputs.counter_keys(p, n)
            wk, wv = oracle.lsd_sort(keys, np.arange(n, dtype=np.uint32))
            assert np.array_equal(to_host(k)[:n], wk), (n, p.dist)
            assert np.array_equal(to_host(v)[:n], wv), (n, p.dist)
        p50, p99, gk, done, peak = srv.stats()
        assert done == len(sizes) and p99 >= p50 > 0 and gk > 0
        assert 0 < peak <= 64 << 20


def test_caller_arrays_sorted_in_place():
    rng = np.random.default_rng(6)
    announce("server caller-owned arrays")
    with Server(hbm_budget_bytes=32 << 20, max_active=16) as srv:
        cases = []
        for i, n in enumerate([5, 16384, 16385, 70_000, 1000, 250_000]):
            keys = inputs.and_keys(n, 4, 40 + i) if i % 2 else inputs.uniform_keys(n, 40 + i)
            vals = inputs.index_values(n)
            kd, vd = to_dev(keys), to_dev(vals)
            cases.append((srv.submit(kd, vd), keys, vals, kd, vd))
        for t, keys, vals, kd, vd in cases:
            srv.wait(t)
            wk, wv = oracle.lsd_sort(keys, vals)
            assert np.array_equal(to_host(kd), wk) and np.array_equal(to_host(vd), wv)
        with pytest.raises(RtError) as e:
            srv.wait(cases[0][0])  # collected by the first wait
        assert e.value.status == RT_ERR_NOT_FOUND


@pytest.mark.parametrize("with_values", [True, False])
def test_caller_arrays_sorted_out_of_place(with_values):
    """Requests with output arrays: each result lands in its outputs, equal
    to the oracle's sort of that input alone, and the inputs are untouched
    (small and tiled requests in one mix; a server serves pairs or keys
    only, not both)."""
    import torch
    announce(f"server caller-owned arrays, out of place, values={with_values}")
    with Server(hbm_budget_bytes=32 << 20, max_active=16) as srv:
        cases = []
        for i, n in enumerate([3, 16384, 16385, 70_000, 250_000, 1000]):
            keys = inputs.zipf16_keys(n, 70 + i) if i % 2 else inputs.uniform_keys(n, 70 + i)
            vals = inputs.index_values(n) if with_values else None
            kd, vd = to_dev(keys), (to_dev(vals) if vals is not None else None)
            ok = torch.empty_like(kd)
            ov = torch.empty_like(vd) if vd is not None else None
            cases.append((srv.submit(kd, vd, ok, ov), keys, vals, kd, vd, ok, ov))
        for t, keys, vals, kd, vd, ok, ov in cases:
            srv.wait(t)
            wk, wv = oracle.lsd_sort(keys, vals)
            assert np.array_equal(to_host(ok), wk), len(keys)
            if vals is not None:
                assert np.array_equal(to_host(ov), wv), len(keys)
                assert np.array_equal(to_host(vd), vals)
            assert np.array_equal(to_host(kd), keys)  # the input is only read


def test_many_long_requests_in_xcd_chunks():
    """At least 128 tiled requests of 16 tiles or more in flight: a step's
    tile list is cut into XCD chunks at request ends.  Every result is the
    oracle's, keys uniform and low-entropy alike."""
    announce("server long requests in XCD chunks")
    rng = np.random.default_rng(11)
    sizes = [int(x) for x in rng.integers(262_144, 360_000, size=136)]
    staged = []  # device copies first, so that the submissions follow each other closely
    for i, n in enumerate(sizes):
        keys = inputs.and_keys(n, 4, 60 + i) if i % 3 == 0 else inputs.uniform_keys(n, 60 + i)
        vals = inputs.index_values(n)
        staged.append((keys, vals, to_dev(keys), to_dev(vals)))
    sync()
    with Server(hbm_budget_bytes=2 << 30, max_active=160) as srv:
        cases = [(srv.submit(kd, vd), keys, vals, kd, vd) for keys, vals, kd, vd in staged]
        for t, keys, vals, kd, vd in cases:
            srv.wait(t)
            wk, wv = oracle.lsd_sort(keys, vals)
            assert np.array_equal(to_host(kd), wk) and np.array_equal(to_host(vd), wv)


def test_budget_admission_waits_and_rejects():
    import torch
    announce("server budget")
    n = 300_000  # generated, pairs: 4 arrays of 1.2 MB
    with Server(hbm_budget_bytes=6 << 20, max_active=8) as srv:
        with pytest.raises(RtError) as e:
            srv.submit_generated(gen_params_to_c(inputs.counter_params(0, 1, 0)), 1 << 20)
        assert e.value.status == RT_ERR_BUDGET
        ts = [(_generated_case(srv, i, n, 0)) for i in range(4)]
        for t, p in ts:
            srv.wait(t)
            k = torch.empty(n, dtype=torch.int32, device="cuda")
            srv.fetch(t, k, None)
            sync()
            assert np.array_equal(to_host(k), np.sort(inputs.counter_keys(p, n)))
        assert srv.stats()[4] <= 6 << 20


def test_cancel_queued_and_admitted_requests():
    """Cancelled requests end as RT_ERR_CANCELLED and leave their arrays
    holding a permutation of the input with every key still beside its own
    value (untouched, or the state after an even number of passes); a
    cancel that comes too late is refused and that result is the oracle's;
    every other request is the oracle's, and the server goes on serving.
    One request is admitted at a time (max_active 1) and the first is 2^26
    pairs, so the requests behind it are still queued when they are
    cancelled right after submission."""
    announce("server cancel")
    sizes = [1 << 26, 2 << 20, 70_000, 2 << 20, 1000, 2 << 20, 300_001]
    data = []
    for i, n in enumerate(sizes):
        keys = inputs.uniform_keys(n, 60 + i)
        vals = inputs.index_values(n)
        data.append((keys, vals, to_dev(keys), to_dev(vals)))
    sync()
    with Server(hbm_budget_bytes=600 << 20, max_active=1) as srv:
        cases = [[srv.submit(kd, vd), keys, vals, kd, vd, None] for keys, vals, kd, vd in data]
        for c in cases[1::2] + [cases[0]]:   # queued ones, then the admitted first one
            try:
                srv.cancel(c[0])
                c[5] = "cancelled"
            except RtError as e:
                assert e.status == RT_ERR_INVALID_ARG   # finished, or its last pass under way
                c[5] = "too late"
        assert sum(c[5] == "cancelled" for c in cases[1::2]) >= 1
        late_keys, late_vals = inputs.uniform_keys(123_457, 69), inputs.index_values(123_457)
        late_kd, late_vd = to_dev(late_keys), to_dev(late_vals)   # kept alive until its wait
        late = srv.submit(late_kd, late_vd)
        for t, keys, vals, kd, vd, what in cases:
            try:
                srv.wait(t)
                status = 0
            except RtError as e:
                status = e.status
            hk, hv = to_host(kd), to_host(vd)
            if what == "cancelled":
                assert status == RT_ERR_CANCELLED, (len(keys), status)
                counts = np.bincount(hv, minlength=len(vals))    # values are the indices
                assert len(counts) == len(vals) and (counts == 1).all(), "a permutation of the input"
                assert np.array_equal(hk, keys[hv]), "every key beside its own value"
            else:
                assert status == 0, (len(keys), status)
                wk, wv = oracle.lsd_sort(keys, vals)
                assert np.array_equal(hk, wk) and np.array_equal(hv, wv)
        srv.wait(late)
        wk, wv = oracle.lsd_sort(late_keys, late_vals)
        assert np.array_equal(to_host(late_kd), wk) and np.array_equal(to_host(late_vd), wv)
        with pytest.raises(RtError) as e:
            srv.cancel(late)                     # collected
        assert e.value.status == RT_ERR_NOT_FOUND


def test_keys_only_server():
    announce("server keys only")
    with Server(hbm_budget_bytes=16 << 20, max_active=8) as srv:
        cases = []
        for i, n in enumerate([3, 9000, 40_000]):
            keys = inputs.uniform_keys(n, 60 + i)
            kd = to_dev(keys)
            cases.append((srv.submit(kd), keys, kd))
        for t, keys, kd in cases:
            srv.wait(t)
            assert np.array_equal(to_host(kd), np.sort(keys))


def test_wait_any_reports_each_request_once_in_completion_order():
    import torch
    announce("server wait_any")
    sizes = [100, 300_000, 5000, 20_000, 3, 70_000, 16385, 2]
    with Server(hbm_budget_bytes=64 << 20, max_active=32) as srv:
        tickets = {}
        for rid, n in enumerate(sizes):
            t, p = _generated_case(srv, 100 + rid, n, rid % 3)
            tickets[t] = (p, n)
        seen = []
        while len(seen) < len(sizes):
            t, lat = srv.wait_any()
            assert t in tickets and t not in seen and lat >= 0
            seen.append(t)
            p, n = tickets[t]
            k = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            srv.fetch(t, k, None)
            sync()
            assert np.array_equal(to_host(k)[:n], np.sort(inputs.counter_keys(p, n)))
        with pytest.raises(RtError) as e:
            srv.wait_any(timeout_us=0)
        assert e.value.status == RT_ERR_NOT_FOUND


def _trace(count, seed, max_log2=16, span_s=0.05):
    import ctypes
    rng = np.random.default_rng(seed)
    arrivals = np.sort(rng.uniform(0, span_s, size=count))
    sizes = np.floor(2.0 ** rng.uniform(0, max_log2, size=count)).astype(np.uint64)
    params = []
    for i in range(count):
        params.append(gen_params_to_c(inputs.counter_params(i % 3, inputs.SEED_SERVING, 900 + i)))
    return arrivals, sizes, params


def test_replay_open_loop_trace():
    """The native open-loop replay submits every request of a trace, and
    each latency (completion - scheduled arrival) is non-negative; the
    server is left with nothing outstanding."""
    announce("server replay of a 300-request trace")
    arrivals, sizes, params = _trace(300, 7)
    with Server(hbm_budget_bytes=64 << 20, max_active=64) as srv:
        lat, span = srv.replay(arrivals, sizes, params)
        assert np.all(lat >= 0), lat[lat < 0][:5]
        assert span >= arrivals[-1] * 1e6
        assert np.all(lat <= span - arrivals * 1e6 + 1.0)
        p50, p99, gk, done, peak = srv.stats()
        assert done == 300
        # nothing left: a second replay on the same server is accepted
        lat2, _ = srv.replay(arrivals[:20], sizes[:20], params[:20])
        assert np.all(lat2 >= 0)


def test_replay_reports_a_refused_submission():
    """A request over the budget stops the submitter; the replay returns
    RT_ERR_BUDGET after the requests already submitted have finished, and
    the refused and later requests have no latency."""
    announce("server replay with a request over the budget")
    arrivals, sizes, params = _trace(40, 8)
    sizes[25] = 1 << 22  # 32 MiB of pairs: over the 8 MiB budget
    with Server(hbm_budget_bytes=8 << 20, max_active=16) as srv:
        with pytest.raises(RtError) as e:
            srv.replay(arrivals, sizes, params)
        assert e.value.status == RT_ERR_BUDGET
        p50, p99, gk, done, peak = srv.stats()
        assert done == 25
