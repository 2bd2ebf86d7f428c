// rt_sched.h -- the serving loop's policy, host code only: admission under
// a device-memory budget, continuous batching at pass granularity, step
// completion and failure, cancellation, collection and latency statistics.
//
// The scheduler knows requests by size and layout, never by their device
// arrays: rt_server.hip turns each planned step into descriptors and
// launches, reports back when the step has run (and whether it failed), and
// holds the lock that serialises every call here.  CPU tests drive the same
// class with a fake executor and a virtual clock.
//
// A step gives every admitted request one unit of work: one counting-sort
// pass over its tiles (a request of more than lds_max items, `passes`
// passes in all) or its whole sort in LDS (at most lds_max items, done in
// its first step).  Requests admitted between two steps join the next one
// at their first pass while the others continue at theirs.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "rtsort.h"

namespace rt {
namespace sched {

constexpr size_t kGranule = 256;

inline size_t round_up(size_t x) { return (x + kGranule - 1) & ~(kGranule - 1); }

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
   public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = round_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }

   private:
    std::map<size_t, size_t> free_;
};

enum State { kQueued, kActive, kDone };

struct Request {
    // set by the submitter
    uint64_t id = 0;
    size_t n = 0;
    bool generated = false;  // the server makes (and keeps) the input
    bool with_values = false;
    // device side, opaque here: the arrays sorted (input, then result), an
    // out-of-place caller input copied into them at admission, the
    // temporaries, the generator's parameters
    uint32_t *k = nullptr, *v = nullptr;
    const uint32_t *in_k = nullptr, *in_v = nullptr;
    uint32_t *tk = nullptr, *tv = nullptr;
    rt_gen_params gen{};
    // set by the scheduler
    size_t data_off = 0, data_bytes = 0;  // arena: generated input/result
    size_t tmp_off = 0, tmp_bytes = 0;    // arena: temporaries
    State state = kQueued;
    rt_status status = RT_OK;
    std::string error;        // detail of a failed request
    uint32_t pass = 0;        // next pass to plan (tiled requests)
    uint32_t row = 0;         // histogram / prefix-sum row
    bool fresh = true;        // no step has touched it yet
    bool planned_out = false; // its last step is planned: nothing left to cancel
    bool cancel = false;      // leaves at the next plan
    bool collected = false;   // reported by a wait
    uint64_t admit_seq = 0;   // admission order
    double t_submit = 0, t_done = 0;
};

// One request's work in a step.
struct StepItem {
    Request *r;
    uint32_t pass;  // the pass it runs (tiled) -- 0 for a whole sort in LDS
    bool fresh;     // first step: input copy/generation and histograms
    bool small;     // sorted whole in LDS in this step
    bool finishes;  // its last pass
};

// A planned step: the work, in descriptor order, and the requests that
// complete when the step has run (its finishing items, and requests that
// leave without work: cancelled, or failed in an earlier step).
struct Step {
    std::vector<StepItem> items;
    std::vector<Request *> finishing;
};

class Scheduler {
   public:
    Scheduler(size_t arena_bytes, uint32_t max_active, uint32_t lds_max, uint32_t passes)
        : arena_bytes_(round_up(arena_bytes)), max_active_(max_active), lds_max_(lds_max), passes_(passes) {
        alloc_.reset(arena_bytes_);
        free_rows_.reserve(max_active);
        for (uint32_t i = max_active; i-- > 0;) free_rows_.push_back(i);
    }

    size_t arena_bytes() const { return arena_bytes_; }
    uint32_t max_active() const { return max_active_; }
    bool is_small(size_t n) const { return n <= lds_max_; }

    // Arena bytes a request holds while admitted: its temporaries when it
    // is tiled, its input/result arrays when the server generates it.
    size_t footprint(size_t n, bool generated, bool with_values) const {
        const size_t arr = round_up(n * sizeof(uint32_t));
        const size_t per = with_values ? 2 : 1;
        return (generated ? per * arr : 0) + (is_small(n) ? 0 : per * arr);
    }

    // Queues a request (the scheduler owns it from now on); returns its id.
    uint64_t submit(std::unique_ptr<Request> r, double now) {
        r->id = next_id_++;
        r->t_submit = now;
        r->state = kQueued;
        if (first_submit_ < 0) first_submit_ = now;
        ++uncollected_;
        queue_.push_back(r.get());
        const uint64_t id = r->id;
        all_[id] = std::move(r);
        return id;
    }

    // The value layout of the requests held (one per server), or -1 if none.
    int held_layout() const {
        for (const auto &kv : all_) return kv.second->with_values ? 1 : 0;
        return -1;
    }

    // Admits queued requests in arrival order while memory and slots last
    // (the head of the queue waits for memory rather than being passed).
    // Returns how many were admitted; appends them to *admitted if given.
    size_t admit(std::vector<Request *> *admitted = nullptr) {
        size_t count = 0;
        while (!queue_.empty() && active_.size() < max_active_) {
            Request *r = queue_.front();
            const size_t arr = round_up(r->n * sizeof(uint32_t));
            const size_t per = r->with_values ? 2 : 1;
            const size_t data_bytes = r->generated ? per * arr : 0;
            const size_t tmp_bytes = is_small(r->n) ? 0 : per * arr;
            size_t data_off = 0, tmp_off = 0;
            if (data_bytes && !alloc_.alloc(data_bytes, &data_off)) break;
            if (tmp_bytes && !alloc_.alloc(tmp_bytes, &tmp_off)) {
                if (data_bytes) alloc_.release(data_off, data_bytes);
                break;
            }
            queue_.pop_front();
            r->data_off = data_off;
            r->data_bytes = data_bytes;
            r->tmp_off = tmp_off;
            r->tmp_bytes = tmp_bytes;
            used_ += data_bytes + tmp_bytes;
            peak_ = std::max(peak_, used_);
            r->row = free_rows_.back();
            free_rows_.pop_back();
            r->state = kActive;
            r->pass = 0;
            r->fresh = true;
            r->admit_seq = admitted_++;
            active_.push_back(r);
            if (admitted) admitted->push_back(r);
            ++count;
        }
        return count;
    }

    bool has_active() const { return !active_.empty(); }
    bool has_queued() const { return !queue_.empty(); }

    // Plans the next step from the admitted requests: every request gets one
    // unit of work, in admission order; a cancelled or failed request leaves
    // without work.  The temporaries and rows of the requests that finish or
    // leave go back to the pools at once: a later step runs after this one
    // (the executor keeps steps in order), so reusing them is ordered behind
    // this step's work.
    void plan(Step &step) {
        step.items.clear();
        step.finishing.clear();
        std::vector<Request *> still;
        for (Request *r : active_) {
            const bool leaves = r->cancel || r->status != RT_OK;
            bool finishes = true;
            if (!leaves) {
                StepItem it{r, 0u, r->fresh, false, false};
                if (r->n < 2) {
                    // nothing to sort: done with this step
                } else if (is_small(r->n)) {
                    it.small = true;
                } else {
                    it.pass = r->pass;
                    finishes = r->pass + 1 == passes_;
                }
                it.finishes = finishes;
                step.items.push_back(it);
                r->fresh = false;
            }
            if (leaves && r->cancel && r->status == RT_OK) {
                r->status = RT_ERR_CANCELLED;
                r->error = "cancelled";
            }
            if (!finishes) {
                ++r->pass;
                still.push_back(r);
                continue;
            }
            r->planned_out = true;
            step.finishing.push_back(r);
            if (r->tmp_bytes) alloc_.release(r->tmp_off, r->tmp_bytes);
            used_ -= r->tmp_bytes;
            r->tmp_bytes = 0;
            free_rows_.push_back(r->row);
        }
        active_.swap(still);
        ++steps_;
    }

    // A planned step has run (status RT_OK) or failed.  A failure marks
    // every request that had work in the step: those that finished with it
    // end failed, the others leave at the next plan, and requests that had
    // no work in it are untouched.
    void complete(Step &step, rt_status status, const std::string &why, double now) {
        if (status != RT_OK)
            for (const StepItem &it : step.items)
                if (it.r->status == RT_OK) {
                    it.r->status = status;
                    it.r->error = why;
                }
        for (Request *r : step.finishing) {
            r->state = kDone;
            r->t_done = now;
            finished_.push_back(r->id);
            if (r->status == RT_OK) {
                latencies_.push_back(now - r->t_submit);
                items_done_ += r->n;
                last_done_ = now;
            }
        }
        step.items.clear();
        step.finishing.clear();
    }

    // Cancels a request: a queued one ends at once (RT_ERR_CANCELLED), an
    // admitted one leaves at the next plan and ends when that step has run
    // (as RT_ERR_CANCELLED, unless a failed step already marked it).
    // RT_ERR_INVALID_ARG when its last step is already planned or it has
    // finished (its result stands); RT_ERR_NOT_FOUND for an unknown or
    // collected ticket.
    rt_status cancel(uint64_t id, double now) {
        auto f = all_.find(id);
        if (f == all_.end() || f->second->collected) return RT_ERR_NOT_FOUND;
        Request *r = f->second.get();
        if (r->state == kQueued) {
            queue_.erase(std::find(queue_.begin(), queue_.end(), r));
            r->status = RT_ERR_CANCELLED;
            r->error = "cancelled";
            r->state = kDone;
            r->t_done = now;
            finished_.push_back(r->id);
            return RT_OK;
        }
        if (r->state == kDone || r->planned_out) return RT_ERR_INVALID_ARG;
        r->cancel = true;
        return RT_OK;
    }

    // Ends every request not yet finished as RT_ERR_CANCELLED (shutdown,
    // after the executor has drained).
    void cancel_all(double now) {
        for (auto &kv : all_) {
            Request *r = kv.second.get();
            if (r->state != kDone) {
                r->state = kDone;
                r->status = RT_ERR_CANCELLED;
                r->error = "server stopped";
                r->t_done = now;
            }
        }
        queue_.clear();
        active_.clear();
    }

    Request *find(uint64_t id) {
        auto f = all_.find(id);
        return f == all_.end() ? nullptr : f->second.get();
    }
    bool done(uint64_t id) const {
        auto f = all_.find(id);
        return f == all_.end() || f->second->state == kDone;
    }
    uint64_t uncollected() const { return uncollected_; }

    // The next finished request no wait has reported (completion order), or
    // 0 if there is none.
    uint64_t next_finished() {
        while (!finished_.empty()) {
            auto f = all_.find(finished_.front());
            if (f != all_.end() && !f->second->collected) return finished_.front();
            finished_.pop_front();
        }
        return 0;
    }

    // Reports a finished request: its status, detail and latency.  A request
    // with nothing left to fetch (not generated) is dropped; a generated one
    // stays until it is fetched or released.
    rt_status collect(uint64_t id, double *latency_us, std::string *why) {
        auto f = all_.find(id);
        if (f == all_.end() || f->second->collected) return RT_ERR_NOT_FOUND;
        Request *r = f->second.get();
        --uncollected_;
        r->collected = true;
        if (latency_us) *latency_us = r->t_done - r->t_submit;
        const rt_status st = r->status;
        if (why) *why = r->error;
        if (!r->generated) drop(f);
        return st;
    }

    // Drops a finished generated request, returning its memory.
    rt_status release(uint64_t id) {
        auto f = all_.find(id);
        if (f == all_.end()) return RT_ERR_NOT_FOUND;
        if (f->second->state != kDone) return RT_ERR_INVALID_ARG;
        drop(f);
        return RT_OK;
    }

    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    uint64_t steps() const { return steps_; }

    // Latency percentiles over completed requests (nearest rank), completed
    // items per second over first submission to last completion.
    void stats(double *p50, double *p99, double *items_per_us, uint64_t *completed) const {
        std::vector<double> l = latencies_;
        std::sort(l.begin(), l.end());
        auto pct = [&](double q) {
            if (l.empty()) return 0.0;
            const size_t i = static_cast<size_t>(q * static_cast<double>(l.size() - 1) + 0.5);
            return l[std::min(i, l.size() - 1)];
        };
        if (p50) *p50 = pct(0.50);
        if (p99) *p99 = pct(0.99);
        if (items_per_us) {
            const double span = last_done_ - first_submit_;
            *items_per_us = (span > 0 && items_done_) ? static_cast<double>(items_done_) / span : 0.0;
        }
        if (completed) *completed = l.size();
    }

   private:
    void drop(std::unordered_map<uint64_t, std::unique_ptr<Request>>::iterator f) {
        Request *r = f->second.get();
        if (r->data_bytes) {
            alloc_.release(r->data_off, r->data_bytes);
            used_ -= r->data_bytes;
            r->data_bytes = 0;
        }
        all_.erase(f);
    }

    size_t arena_bytes_;
    uint32_t max_active_;
    uint32_t lds_max_;
    uint32_t passes_;
    Arena alloc_;
    size_t used_ = 0, peak_ = 0;
    std::deque<Request *> queue_;
    std::vector<Request *> active_;
    std::vector<uint32_t> free_rows_;
    std::deque<uint64_t> finished_;  // tickets in completion order
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all_;
    uint64_t next_id_ = 1;
    uint64_t admitted_ = 0;
    uint64_t uncollected_ = 0;
    uint64_t steps_ = 0;
    std::vector<double> latencies_;
    double first_submit_ = -1, last_done_ = 0;
    uint64_t items_done_ = 0;
};

}  // namespace sched
}  // namespace rt
