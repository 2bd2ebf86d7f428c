"""The serving scheduler's policy on the CPU: the class the server runs
(paper_1008_2849_amd/csrc/rt_sched.h), driven through tests/sched_shim.cpp
with a fake executor (planned steps complete when and how the test says)
and a virtual clock (every time is the test's number).

Covered: FIFO admission under the memory budget and the slot limit,
continuous batching at pass granularity (a tiled request takes exactly one
pass per step, a small one finishes in its first step, latecomers join the
next step at pass 0), memory coming back when requests finish, cancellation
of queued and admitted requests, a failed step failing only the requests that
had work in it, collection and release, shutdown, latency statistics, and a
seeded random workload checked against the invariants.
"""
import ctypes
import os
import random
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RT_OK, RT_ERR_INVALID_ARG, RT_ERR_HIP, RT_ERR_CANCELLED, RT_ERR_NOT_FOUND = 0, 1, 4, 7, 9
QUEUED, ACTIVE, DONE = 0, 1, 2
FRESH, SMALL, FINISHES = 1, 2, 4
LDS_MAX = 16384   # the largest request sorted whole in LDS
PASSES = 4        # passes of a tiled request
MiB = 1 << 20


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = tmp_path_factory.mktemp("sched") / "libsched_shim.so"
    subprocess.run([cxx, "-std=c++17", "-O1", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1008_2849_amd", "csrc"),
                    "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "sched_shim.cpp"), "-o", str(out)],
                   check=True)
    so = ctypes.CDLL(str(out))
    vp, sz, u32, u64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    P = ctypes.POINTER
    for name, res, args in (
            ("sim_new", vp, [sz, u32, u32, u32]), ("sim_free", None, [vp]),
            ("sim_footprint", sz, [vp, sz, ctypes.c_int, ctypes.c_int]),
            ("sim_submit", u64, [vp, sz, ctypes.c_int, ctypes.c_int, dbl]), ("sim_admit", sz, [vp]),
            ("sim_has_active", ctypes.c_int, [vp]),
            ("sim_plan", ctypes.c_int, [vp, P(u64), P(u32), P(u32), ctypes.c_int, P(u64), ctypes.c_int,
                                        P(ctypes.c_int)]),
            ("sim_inflight", ctypes.c_int, [vp]), ("sim_complete", ctypes.c_int, [vp, ctypes.c_int, dbl]),
            ("sim_cancel", ctypes.c_int, [vp, u64, dbl]),
            ("sim_query", ctypes.c_int, [vp, u64, P(ctypes.c_int), P(ctypes.c_int), P(u32), P(u64),
                                         P(ctypes.c_int), P(sz), P(sz)]),
            ("sim_collect", ctypes.c_int, [vp, u64, P(dbl)]), ("sim_next_finished", u64, [vp]),
            ("sim_release", ctypes.c_int, [vp, u64]), ("sim_cancel_all", None, [vp, dbl]),
            ("sim_stats", None, [vp, P(sz), P(sz), P(u64), P(dbl), P(dbl), P(dbl), P(u64)])):
        f = getattr(so, name)
        f.restype = res
        f.argtypes = args
    return so


class Sim:
    """One scheduler with a fake executor."""

    def __init__(self, so, arena, max_active=64):
        self.so = so
        self.h = so.sim_new(arena, max_active, LDS_MAX, PASSES)

    def close(self):
        self.so.sim_free(self.h)

    def footprint(self, n, generated=False, values=True):
        return self.so.sim_footprint(self.h, n, int(generated), int(values))

    def submit(self, n, now, generated=False, values=True):
        return self.so.sim_submit(self.h, n, int(generated), int(values), float(now))

    def admit(self):
        return self.so.sim_admit(self.h)

    def plan(self):
        """Plans a step: ({ticket: (pass, flags)} in item order, [finishing tickets]), or None."""
        cap = 4096
        ids, passes, flags = (ctypes.c_uint64 * cap)(), (ctypes.c_uint32 * cap)(), (ctypes.c_uint32 * cap)()
        fin, nfin = (ctypes.c_uint64 * cap)(), ctypes.c_int()
        n = self.so.sim_plan(self.h, ids, passes, flags, cap, fin, cap, ctypes.byref(nfin))
        if n < 0:
            return None
        return {ids[i]: (passes[i], flags[i]) for i in range(n)}, [fin[i] for i in range(nfin.value)]

    def complete(self, now, status=RT_OK):
        assert self.so.sim_complete(self.h, status, float(now)) == 0

    def cancel(self, t, now):
        return self.so.sim_cancel(self.h, t, float(now))

    def query(self, t):
        st, status, ps, seq, col = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_int()
        tmp, data = ctypes.c_size_t(), ctypes.c_size_t()
        if self.so.sim_query(self.h, t, *(ctypes.byref(x) for x in (st, status, ps, seq, col, tmp, data))) != 0:
            return None
        return dict(state=st.value, status=status.value, pass_=ps.value, seq=seq.value, collected=col.value,
                    tmp=tmp.value, data=data.value)

    def collect(self, t):
        lat = ctypes.c_double()
        st = self.so.sim_collect(self.h, t, ctypes.byref(lat))
        return st, lat.value

    def next_finished(self):
        return self.so.sim_next_finished(self.h)

    def release(self, t):
        return self.so.sim_release(self.h, t)

    def stats(self):
        used, peak, done, unc = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_uint64(), ctypes.c_uint64()
        p50, p99, rate = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self.so.sim_stats(self.h, *(ctypes.byref(x) for x in (used, peak, done, p50, p99, rate, unc)))
        return dict(used=used.value, peak=peak.value, completed=done.value, p50=p50.value, p99=p99.value,
                    rate=rate.value, uncollected=unc.value)

    def step(self, now, status=RT_OK):
        """Admit, plan one step and complete it at `now`; returns the plan."""
        self.admit()
        p = self.plan()
        if p is not None:
            self.complete(now, status)
        return p


@pytest.fixture
def mk(shim):
    made = []

    def make(arena, max_active=64):
        s = Sim(shim, arena, max_active)
        made.append(s)
        return s
    yield make
    for s in made:
        s.close()


def test_footprint(mk):
    s = mk(64 * MiB)
    big = 1 << 20
    assert s.footprint(100) == 0                         # whole in LDS: no temporaries
    assert s.footprint(LDS_MAX + 1) == 2 * ((4 * (LDS_MAX + 1) + 255) // 256 * 256)
    assert s.footprint(big) == 2 * 4 * big               # key and value temporaries
    assert s.footprint(big, values=False) == 4 * big
    assert s.footprint(big, generated=True) == 4 * 4 * big   # plus the generated input/result
    assert s.footprint(100, generated=True) == 2 * 512


def test_pass_granularity_and_latecomers(mk):
    """A tiled request takes one pass per step and finishes after PASSES
    steps; a small one finishes in its first step; a request admitted later
    joins the next step at pass 0 while the first continues at its own."""
    s = mk(256 * MiB)
    a = s.submit(1 << 20, now=0)
    small = s.submit(1000, now=0)
    items, fin = s.step(now=10)
    assert items[a] == (0, FRESH) and items[small] == (0, FRESH | SMALL | FINISHES)
    assert fin == [small] and s.query(small)["state"] == DONE
    b = s.submit(1 << 19, now=11)
    items, fin = s.step(now=20)
    assert items == {a: (1, 0), b: (0, FRESH)} and fin == []
    items, _ = s.step(now=30)
    assert items == {a: (2, 0), b: (1, 0)}
    items, fin = s.step(now=40)
    assert items == {a: (3, FINISHES), b: (2, 0)} and fin == [a]
    items, fin = s.step(now=50)
    assert items == {b: (3, FINISHES)} and fin == [b]
    assert s.plan() is None
    assert s.collect(a) == (RT_OK, 40.0) and s.collect(b) == (RT_OK, 39.0) and s.collect(small) == (RT_OK, 10.0)
    assert s.stats()["used"] == 0 and s.stats()["completed"] == 3


def test_tiny_requests_finish_in_one_step(mk):
    s = mk(16 * MiB)
    t0, t1 = s.submit(0, now=0), s.submit(1, now=0)
    items, fin = s.step(now=1)
    assert items[t0][1] & FINISHES and items[t1][1] & FINISHES and sorted(fin) == sorted([t0, t1])


def test_fifo_admission_under_budget(mk):
    """Admission is first come, first served: the head waits for memory and
    nothing behind it passes it; used memory never exceeds the budget, and
    the queue advances as finished requests give their temporaries back."""
    arena = 64 * MiB
    s = mk(arena)
    n = 3 << 20                          # 24 MiB of temporaries each
    tickets = [s.submit(n, now=i) for i in range(5)]
    assert s.admit() == 2                # 48 MiB of 64
    small = s.submit(100, now=5)         # would fit, but must not pass the queue
    assert s.admit() == 0
    assert [s.query(t)["state"] for t in tickets] == [ACTIVE, ACTIVE, QUEUED, QUEUED, QUEUED]
    assert s.query(small)["state"] == QUEUED
    for now in (10, 20, 30):
        s.step(now)
        assert s.stats()["used"] <= arena
        assert s.query(tickets[2])["state"] == QUEUED
    items, fin = s.step(now=40)          # the first two finish; their memory returns at planning
    assert sorted(fin) == tickets[:2]
    assert s.admit() == 2                # the next two fit now, then the small one waits behind the fifth
    assert s.query(tickets[4])["state"] == QUEUED and s.query(small)["state"] == QUEUED
    seqs = [s.query(t)["seq"] for t in tickets[:4]]
    assert seqs == sorted(seqs)
    assert s.stats()["peak"] <= arena


def test_slot_limit(mk):
    s = mk(1 << 30, max_active=3)
    tickets = [s.submit(1 << 16, now=0) for _ in range(5)]
    assert s.admit() == 3
    assert [s.query(t)["state"] for t in tickets] == [ACTIVE] * 3 + [QUEUED] * 2


def test_cancel_queued(mk):
    """A queued request cancelled ends at once, never reaches a step, and
    its wait reports RT_ERR_CANCELLED."""
    s = mk(32 * MiB)
    first = s.submit(3 << 20, now=0)     # 24 MiB: the second cannot be admitted beside it
    second = s.submit(3 << 20, now=1)
    s.admit()
    assert s.query(second)["state"] == QUEUED
    assert s.cancel(second, now=2) == RT_OK
    assert s.query(second)["state"] == DONE and s.query(second)["status"] == RT_ERR_CANCELLED
    assert s.next_finished() == second
    assert s.collect(second) == (RT_ERR_CANCELLED, 1.0)
    for now in (10, 20, 30, 40):
        items, _ = s.step(now)
        assert second not in items
    assert s.collect(first)[0] == RT_OK
    assert s.cancel(second, now=50) == RT_ERR_NOT_FOUND   # collected


def test_cancel_admitted(mk):
    """An admitted request cancelled takes no further pass, gives back its
    memory at the next plan and ends with that step; the others go on
    untouched."""
    s = mk(256 * MiB)
    keep = s.submit(1 << 20, now=0)
    drop = s.submit(1 << 21, now=0)
    s.step(now=10)
    used_before = s.stats()["used"]
    assert s.cancel(drop, now=11) == RT_OK
    assert s.query(drop)["state"] == ACTIVE
    s.admit()
    items, fin = s.plan()
    assert drop not in items and drop in fin and items[keep] == (1, 0)
    assert s.stats()["used"] == used_before - s.footprint(1 << 21)
    s.complete(now=20)
    assert s.query(drop)["status"] == RT_ERR_CANCELLED
    s.step(now=30)
    s.step(now=40)
    assert s.collect(keep)[0] == RT_OK and s.collect(drop)[0] == RT_ERR_CANCELLED
    st = s.stats()
    assert st["completed"] == 1 and st["used"] == 0


def test_cancel_too_late(mk):
    """Once a request's last pass is planned, cancelling is refused and its
    result stands; cancelling a finished one is refused too."""
    s = mk(256 * MiB)
    t = s.submit(1 << 20, now=0)
    small = s.submit(10, now=0)
    s.step(now=1)
    assert s.cancel(small, now=2) == RT_ERR_INVALID_ARG      # sorted in its first step
    for now in (10, 20):
        s.step(now)
    s.admit()
    items, fin = s.plan()                                     # the last pass, in flight
    assert items[t] == (3, FINISHES)
    assert s.cancel(t, now=25) == RT_ERR_INVALID_ARG
    s.complete(now=30)
    assert s.collect(t)[0] == RT_OK
    assert s.cancel(12345, now=31) == RT_ERR_NOT_FOUND


def test_cancel_before_first_step(mk):
    """Admitted but not yet in a step: it leaves without any work."""
    s = mk(256 * MiB)
    t = s.submit(1 << 20, now=0)
    s.admit()
    assert s.cancel(t, now=1) == RT_OK
    items, fin = s.plan()
    assert items == {} and fin == [t]
    s.complete(now=2)
    assert s.collect(t)[0] == RT_ERR_CANCELLED and s.stats()["used"] == 0


def test_failed_step_isolation(mk):
    """A failed step fails the requests that had work in it: the ones that
    finished with it end failed, the others leave at the next plan with
    their memory returned; a request admitted after the failure is untouched
    and the scheduler keeps serving."""
    s = mk(256 * MiB)
    a = s.submit(1 << 20, now=0)
    b = s.submit(1 << 19, now=0)
    s.step(now=10)
    s.step(now=20)
    s.admit()
    items, _ = s.plan()
    assert set(items) == {a, b}
    later = s.submit(1 << 18, now=21)    # submitted while the failing step runs
    s.complete(now=30, status=RT_ERR_HIP)
    assert s.query(a)["status"] == RT_ERR_HIP and s.query(b)["status"] == RT_ERR_HIP
    s.admit()
    items, fin = s.plan()
    assert set(items) == {later} and sorted(fin) == sorted([a, b])
    assert s.stats()["used"] == s.footprint(1 << 18)
    s.complete(now=40)
    for now in (50, 60, 70):
        s.step(now)
    assert s.collect(a)[0] == RT_ERR_HIP and s.collect(b)[0] == RT_ERR_HIP
    assert s.collect(later) == (RT_OK, 49.0)
    assert s.stats()["completed"] == 1 and s.stats()["used"] == 0


def test_cancel_after_a_failed_step(mk):
    """A request a failed step has marked can still be cancelled (it takes no
    further pass either way) and ends with the step's failure."""
    s = mk(256 * MiB)
    t = s.submit(1 << 20, now=0)
    s.step(now=1)
    s.step(now=2, status=RT_ERR_HIP)
    assert s.query(t)["state"] == ACTIVE and s.query(t)["status"] == RT_ERR_HIP
    assert s.cancel(t, now=3) == RT_OK
    items, fin = s.step(now=4)
    assert items == {} and fin == [t]
    assert s.collect(t)[0] == RT_ERR_HIP


def test_failed_final_step(mk):
    """A request whose last step fails ends failed, not OK."""
    s = mk(64 * MiB)
    t = s.submit(1000, now=0)
    s.step(now=5, status=RT_ERR_HIP)
    assert s.query(t)["state"] == DONE and s.collect(t)[0] == RT_ERR_HIP
    assert s.stats()["completed"] == 0


def test_generated_results_held_until_release(mk):
    """A generated request keeps its input/result memory after its wait
    until it is released; collecting twice is refused."""
    s = mk(256 * MiB)
    t = s.submit(1 << 20, now=0, generated=True)
    for now in (1, 2, 3, 4):
        s.step(now)
    assert s.stats()["used"] == 8 * MiB                    # keys and values stay
    assert s.collect(t) == (RT_OK, 4.0)
    assert s.collect(t)[0] == RT_ERR_NOT_FOUND
    assert s.release(t) == RT_OK and s.stats()["used"] == 0
    assert s.release(t) == RT_ERR_NOT_FOUND


def test_release_unfinished_refused(mk):
    s = mk(256 * MiB)
    t = s.submit(1 << 20, now=0, generated=True)
    s.step(now=1)
    assert s.release(t) == RT_ERR_INVALID_ARG


def test_completion_order(mk):
    """next_finished reports requests in completion order, each once."""
    s = mk(256 * MiB)
    big = s.submit(1 << 20, now=0)
    small = s.submit(100, now=0)
    s.step(now=1)
    assert s.next_finished() == small
    s.collect(small)
    assert s.next_finished() == 0
    for now in (2, 3, 4):
        s.step(now)
    assert s.next_finished() == big


def test_shutdown_cancels_the_rest(mk):
    s = mk(32 * MiB)
    a = s.submit(1 << 20, now=0)
    b = s.submit(3 << 20, now=0)
    c = s.submit(3 << 20, now=0)
    s.step(now=1)
    s.so.sim_cancel_all(s.h, 2.0)
    for t in (a, b, c):
        assert s.query(t)["state"] == DONE and s.query(t)["status"] == RT_ERR_CANCELLED


def test_latency_statistics(mk):
    """Percentiles by nearest rank over the completed requests' latencies on
    the virtual clock; the rate is items over first submission to last
    completion."""
    s = mk(1 << 30)
    lat = []
    for i in range(100):
        s.submit(100, now=float(i))
        s.step(now=float(i) + 1 + i % 7)
        lat.append(1 + i % 7)
    st = s.stats()
    lat.sort()
    assert st["completed"] == 100
    assert st["p50"] == lat[round(0.5 * 99)] and st["p99"] == lat[round(0.99 * 99)]
    assert st["rate"] == pytest.approx(100 * 100 / (99 + 1 + 99 % 7))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_workload_invariants(mk, seed):
    """Random arrivals, sizes, cancellations and step failures (seeded):
    used memory stays within the budget, admission follows submission order,
    every request ends exactly once with a consistent status, a request that
    ends OK took exactly its passes, and all memory returns at the end."""
    rng = random.Random(seed)
    arena = 96 * MiB
    s = mk(arena, max_active=16)
    passes_seen = {}
    status_of = {}
    submitted = []
    now = 0.0
    for step in range(400):
        for _ in range(rng.randrange(3)):
            n = int(2 ** rng.uniform(6, 22))
            t = s.submit(n, now, generated=rng.random() < 0.3)
            submitted.append((t, n))
        if submitted and rng.random() < 0.1:
            t, _ = rng.choice(submitted)
            r = s.cancel(t, now)
            assert r in (RT_OK, RT_ERR_INVALID_ARG, RT_ERR_NOT_FOUND)
        s.admit()
        plan = s.plan()
        if plan is not None:
            items, fin = plan
            for t, (p, fl) in items.items():
                if not fl & SMALL:
                    assert p == passes_seen.get(t, 0), "passes run in order, one per step"
                passes_seen[t] = passes_seen.get(t, 0) + 1
            s.complete(now + 1, RT_ERR_HIP if rng.random() < 0.03 else RT_OK)
        assert s.stats()["used"] <= arena
        while True:
            t = s.next_finished()
            if not t:
                break
            st, _ = s.collect(t)
            assert t not in status_of
            status_of[t] = st
            if st == RT_OK:
                n = dict(submitted)[t]
                if n >= 2:
                    assert passes_seen[t] == (1 if n <= LDS_MAX else PASSES)
            if s.query(t) is not None:       # a generated request: release it
                assert s.release(t) == RT_OK
        now += 1.0
    # drain
    for _ in range(2000):
        if s.stats()["uncollected"] == 0:
            break
        s.admit()
        if s.plan() is not None:
            s.complete(now)
        while True:
            t = s.next_finished()
            if not t:
                break
            status_of[t] = s.collect(t)[0]
            if s.query(t) is not None:
                s.release(t)
        now += 1.0
    assert len(status_of) == len(submitted)
    assert set(status_of.values()) <= {RT_OK, RT_ERR_HIP, RT_ERR_CANCELLED}
    assert s.stats()["used"] == 0
