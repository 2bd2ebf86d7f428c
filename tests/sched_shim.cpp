// A C interface over the serving scheduler (paper_1008_2849_amd/csrc/rt_sched.h)
// with a fake executor: planned steps wait in a FIFO until the test
// completes them, successfully or not, at a time the test chooses (a virtual
// clock).  Built with the host compiler by tests/test_sched.py; no device
// code is involved.
#include <cstring>
#include <deque>
#include <memory>

#include "rt_sched.h"

using rt::sched::Request;
using rt::sched::Scheduler;
using rt::sched::Step;

namespace {
struct Sim {
    Sim(size_t arena, uint32_t max_active, uint32_t lds_max, uint32_t passes)
        : s(arena, max_active, lds_max, passes) {}
    Scheduler s;
    std::deque<Step> inflight;  // planned, not yet completed (oldest first)
};
Sim *sim(void *p) { return static_cast<Sim *>(p); }
}  // namespace

extern "C" {

void *sim_new(size_t arena, uint32_t max_active, uint32_t lds_max, uint32_t passes) {
    return new Sim(arena, max_active, lds_max, passes);
}

void sim_free(void *p) { delete sim(p); }

size_t sim_footprint(void *p, size_t n, int generated, int with_values) {
    return sim(p)->s.footprint(n, generated != 0, with_values != 0);
}

uint64_t sim_submit(void *p, size_t n, int generated, int with_values, double now) {
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->generated = generated != 0;
    r->with_values = with_values != 0;
    return sim(p)->s.submit(std::move(r), now);
}

size_t sim_admit(void *p) { return sim(p)->s.admit(); }

int sim_has_active(void *p) { return sim(p)->s.has_active() ? 1 : 0; }

// Plans the next step.  Writes each item's ticket, pass and flags (bit 0
// fresh, bit 1 whole in LDS, bit 2 finishes) and the tickets of the
// requests that complete with the step; returns the item count, or -1 when
// nothing is admitted (no step is planned then).
int sim_plan(void *p, uint64_t *ids, uint32_t *passes, uint32_t *flags, int cap, uint64_t *fin, int fcap,
             int *nfin) {
    Sim *m = sim(p);
    if (!m->s.has_active()) return -1;
    m->inflight.emplace_back();
    Step &st = m->inflight.back();
    m->s.plan(st);
    const int n = static_cast<int>(st.items.size());
    for (int i = 0; i < n && i < cap; ++i) {
        ids[i] = st.items[i].r->id;
        passes[i] = st.items[i].pass;
        flags[i] = (st.items[i].fresh ? 1u : 0u) | (st.items[i].small ? 2u : 0u) | (st.items[i].finishes ? 4u : 0u);
    }
    *nfin = static_cast<int>(st.finishing.size());
    for (int i = 0; i < *nfin && i < fcap; ++i) fin[i] = st.finishing[i]->id;
    return n;
}

int sim_inflight(void *p) { return static_cast<int>(sim(p)->inflight.size()); }

// Completes the oldest planned step with `status` (RT_OK or a failure).
int sim_complete(void *p, int status, double now) {
    Sim *m = sim(p);
    if (m->inflight.empty()) return -1;
    m->s.complete(m->inflight.front(), static_cast<rt_status>(status), status ? "injected failure" : "", now);
    m->inflight.pop_front();
    return 0;
}

int sim_cancel(void *p, uint64_t id, double now) { return sim(p)->s.cancel(id, now); }

// State of a request: 0 if known (state 0 queued, 1 admitted, 2 done), -1 if not.
int sim_query(void *p, uint64_t id, int *state, int *status, uint32_t *pass, uint64_t *admit_seq, int *collected,
              size_t *tmp_bytes, size_t *data_bytes) {
    const Request *r = sim(p)->s.find(id);
    if (r == nullptr) return -1;
    *state = static_cast<int>(r->state);
    *status = static_cast<int>(r->status);
    *pass = r->pass;
    *admit_seq = r->admit_seq;
    *collected = r->collected ? 1 : 0;
    *tmp_bytes = r->tmp_bytes;
    *data_bytes = r->data_bytes;
    return 0;
}

int sim_collect(void *p, uint64_t id, double *latency) { return sim(p)->s.collect(id, latency, nullptr); }

uint64_t sim_next_finished(void *p) { return sim(p)->s.next_finished(); }

int sim_release(void *p, uint64_t id) { return sim(p)->s.release(id); }

void sim_cancel_all(void *p, double now) { sim(p)->s.cancel_all(now); }

void sim_stats(void *p, size_t *used, size_t *peak, uint64_t *completed, double *p50, double *p99,
               double *items_per_us, uint64_t *uncollected) {
    const Scheduler &s = sim(p)->s;
    *used = s.used();
    *peak = s.peak();
    s.stats(p50, p99, items_per_us, completed);
    *uncollected = s.uncollected();
}

}  // extern "C"
