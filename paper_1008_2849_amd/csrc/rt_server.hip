// rt_server.hip -- the serving loop: requests to sort arrive one by one, are
// admitted under a device-memory budget, and progress together in steps.
//
// Continuous batching at pass granularity: every step runs, for every
// admitted request, one counting-sort pass over its tiles (requests of more
// than 16K items) or its whole sort in LDS (smaller ones), all in the same
// few launches of the segmented kernels.  A request admitted between two
// steps joins the next one: its input is generated (for generated
// requests), its digit histograms and prefix sums are built at the start of
// that step, and its first pass runs in it.  A request of more than 16K
// items is done after four steps, a smaller one after one.
//
// The policy (admission, which request runs which pass, completion,
// cancellation, failures) is the host-only scheduler of rt_sched.h, called
// under the server's lock.  This file is its device side: the scheduler
// thread turns each planned step into descriptors and work lists, uploads
// them from pinned memory, enqueues the step's kernels on the server's
// stream and records an event; a request is reported done when the event
// of its last step has fired.  Up to `depth` steps may be in flight
// (RT_SERVER_DEPTH, default 1: requests that arrive during a step then join
// the very next one, which measured best for latency and throughput).
//
// Memory: one arena of hbm_budget_bytes, carved first-fit (256-byte
// granules) into each request's temporaries (and, for generated requests,
// its input/result arrays).  Fixed metadata besides the arena: per-request
// histogram and prefix-sum rows, descriptors, work lists and the lookback
// words of one step.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rt_common.h"
#include "rt_sched.h"
#include "rt_seg_kernels.h"

namespace rt {
namespace {

using Clock = std::chrono::steady_clock;

double now_us() {
    return std::chrono::duration<double, std::micro>(Clock::now().time_since_epoch()).count();
}

constexpr size_t kMaxRequestItems = (static_cast<size_t>(1) << 30) - 1;  // 32-bit lookback words

using sched::Request;
using sched::round_up;

// One generated request of a step: its arrays and stream parameters.
struct GenDesc {
    uint32_t *k, *v;
    uint32_t n;
    uint32_t first_chunk;  // chunks of the step's generated requests before this one
    GenArgs g;
};
constexpr uint32_t kGenChunk = 4096;  // items per generating block

// Device metadata of one step: [header | descs | lists | first_tile |
// tile_seg] for the pass work, a second header/list/first_tile/tile_seg set
// for the histogram work of fresh requests, the per-request rows and the
// lookback words.  The leading "step block" (headers, descs, lists) is
// uploaded from pinned host memory once per step.
struct Meta {
    size_t hdr_pass, hdr_hist, descs, lists_pass, list_hist, block_bytes, gen;
    size_t first_pass, first_hist, seg_pass, seg_hist, hist, base, status, total;
    uint32_t max_tiles;
};

Meta make_meta(uint32_t max_active, size_t arena_bytes, uint32_t lds_max) {
    Meta m{};
    auto a = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
    // A tiled request (n > L = lds_max items) holds at least 4n bytes of
    // arena and has ceil(n / 16K) <= n / 16K + 1 < n / 16K + n / L tiles, so
    // a step has at most min(arena / 64K + arena / 4L, arena / 64K +
    // max_active) tiles.
    const size_t by_size = arena_bytes / (sizeof(uint32_t) * kSegTile) +
                           arena_bytes / (sizeof(uint32_t) * (static_cast<size_t>(lds_max) + 1));
    const size_t by_count = arena_bytes / (sizeof(uint32_t) * kSegTile) + max_active;
    m.max_tiles = static_cast<uint32_t>(std::min(by_size, by_count) + 1);
    size_t off = 0;
    m.hdr_pass = off;   off += a(sizeof(SegHeader));
    m.hdr_hist = off;   off += a(sizeof(SegHeader));
    m.descs = off;      off += a(sizeof(SegDesc) * max_active);
    m.lists_pass = off; off += a(sizeof(uint32_t) * (kSegMaxClasses + 1) * max_active);
    m.list_hist = off;  off += a(sizeof(uint32_t) * (kSegMaxClasses + 1) * max_active);
    m.block_bytes = off;
    m.gen = off;        off += a(sizeof(GenDesc) * max_active);
    m.first_pass = off; off += a(sizeof(uint32_t) * (max_active + 1));
    m.first_hist = off; off += a(sizeof(uint32_t) * (max_active + 1));
    m.seg_pass = off;   off += a(sizeof(SegDesc) * m.max_tiles);
    m.seg_hist = off;   off += a(sizeof(SegDesc) * m.max_tiles);
    m.hist = off;       off += a(sizeof(uint32_t) * kSegPasses * kSegRadix * max_active);
    m.base = off;       off += a(sizeof(uint32_t) * kSegPasses * kSegRadix * max_active);
    m.status = off;     off += a(sizeof(uint32_t) * kSegRadix * static_cast<size_t>(m.max_tiles));
    m.total = off;
    return m;
}

// Fills the inputs of every generated request of a step.  The requests'
// items are cut into chunks of kGenChunk, numbered across the requests in
// order; block b fills chunk b (found by binary search over first_chunk).
__global__ __launch_bounds__(256) void k_srv_generate(const GenDesc *__restrict__ gd, uint32_t count) {
    uint32_t lo = 0, hi = count - 1;  // the last request with first_chunk <= b
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) / 2;
        if (gd[mid].first_chunk <= blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const GenDesc &d = gd[lo];
    const uint32_t begin = (blockIdx.x - d.first_chunk) * kGenChunk;
    const uint32_t end = min(d.n, begin + kGenChunk);
    for (uint32_t i = begin + threadIdx.x; i < end; i += 256) {
        d.k[i] = generate_key(d.g, i);
        if (d.v) d.v[i] = i;
    }
}

// Zeroes the histogram rows of the listed (fresh) requests.
__global__ __launch_bounds__(256) void k_srv_clear_rows(const SegDesc *__restrict__ descs,
                                                        const uint32_t *__restrict__ list,
                                                        const SegHeader *__restrict__ h, uint32_t *__restrict__ hist) {
    const uint32_t count = h->count[kSegLarge];
    for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
        uint32_t *row = hist + static_cast<size_t>(descs[list[e]].row) * kSegPasses * kSegRadix;
        for (uint32_t i = threadIdx.x; i < kSegPasses * kSegRadix; i += 256) row[i] = 0u;
    }
}

}  // namespace
}  // namespace rt

using namespace rt;

constexpr int kRing = 8;  // most steps in flight (ring slots)

// Host side of one step in flight: its pinned staging (step block, then the
// generated-request descriptors, then the header words read back), the
// event that marks its end, the scheduler's plan of it, and a failure to
// enqueue it.
struct StepSlot {
    char *host = nullptr;
    hipEvent_t done = nullptr;
    sched::Step step;
    rt_status enqueue_status = RT_OK;
    std::string enqueue_error;
};

struct rt_server {
    int device = 0;
    hipStream_t stream = nullptr;  // every step, in order
    hipStream_t io = nullptr;      // fetch copies
    char *arena = nullptr;
    size_t arena_bytes = 0;
    uint32_t max_active = 0;
    rt::SegClassTable classes{};  // whole-in-LDS size classes, fixed at creation
    Meta meta{};
    char *dmeta = nullptr;
    StepSlot ring[kRing];
    int depth = 1;       // steps in flight at most (1..kRing); 1 measured best
    int ring_head = 0;   // oldest step in flight
    int ring_count = 0;  // steps in flight

    std::mutex mu;  // guards sched, stop and the ring bookkeeping
    std::condition_variable cv_work, cv_done;
    std::unique_ptr<sched::Scheduler> sched;
    bool stop = false;
    std::thread thr;
};

namespace {

size_t slot_bytes(const Meta &m, uint32_t max_active) {
    return m.block_bytes + sizeof(GenDesc) * max_active + 2 * 256;
}

// Points newly admitted requests at their arena ranges (mu held).
void place(rt_server *s, const std::vector<Request *> &admitted) {
    for (Request *r : admitted) {
        const size_t arr = round_up(r->n * sizeof(uint32_t));
        if (r->generated) {
            r->k = reinterpret_cast<uint32_t *>(s->arena + r->data_off);
            r->v = r->with_values ? reinterpret_cast<uint32_t *>(s->arena + r->data_off + arr) : nullptr;
        }
        if (r->tmp_bytes) {
            r->tk = reinterpret_cast<uint32_t *>(s->arena + r->tmp_off);
            r->tv = r->with_values ? reinterpret_cast<uint32_t *>(s->arena + r->tmp_off + arr) : nullptr;
        }
    }
}

// Builds the next step in ring slot `slot` (mu held): the scheduler plans
// it (one pass, or the whole sort in LDS, for every admitted request), then
// its descriptors and work lists are written to the slot's pinned block.
struct StepPlan {
    size_t tiles = 0;
    uint32_t fresh_tiled = 0, tiled = 0, small[kSegMaxClasses] = {0, 0, 0, 0}, gen = 0, gen_chunks = 0;
    bool vals = false;
    // device copies of out-of-place inputs into their outputs: (dst, src, bytes)
    std::vector<std::tuple<void *, const void *, size_t>> copies;
};

StepPlan build_step(rt_server *s, StepSlot &slot) {
    const Meta &m = s->meta;
    StepPlan P;
    s->sched->plan(slot.step);
    slot.enqueue_status = RT_OK;
    slot.enqueue_error.clear();
    char *hb = slot.host;
    memset(hb, 0, m.block_bytes);
    SegHeader *hp = reinterpret_cast<SegHeader *>(hb + m.hdr_pass);
    SegHeader *hh = reinterpret_cast<SegHeader *>(hb + m.hdr_hist);
    SegDesc *descs = reinterpret_cast<SegDesc *>(hb + m.descs);
    uint32_t *lists = reinterpret_cast<uint32_t *>(hb + m.lists_pass);
    uint32_t *hlist = reinterpret_cast<uint32_t *>(hb + m.list_hist) + static_cast<size_t>(kSegLarge) * s->max_active;
    GenDesc *gen = reinterpret_cast<GenDesc *>(hb + m.block_bytes);
    const uint32_t stride = s->max_active;
    const auto &items = slot.step.items;
    for (size_t i = 0; i < items.size(); ++i) {
        const sched::StepItem &it = items[i];
        const Request *r = it.r;
        P.vals = P.vals || r->with_values;
        SegDesc &d = descs[i];
        d.k = r->k;
        d.v = r->with_values ? r->v : nullptr;
        d.tk = r->tk;
        d.tv = r->with_values ? r->tv : nullptr;
        d.n = static_cast<uint32_t>(r->n);
        d.pass = it.pass;
        d.row = r->row;
        if (it.fresh && r->in_k != nullptr && r->n > 0) {
            P.copies.emplace_back(r->k, r->in_k, r->n * sizeof(uint32_t));
            if (r->with_values) P.copies.emplace_back(r->v, r->in_v, r->n * sizeof(uint32_t));
        }
        if (it.fresh && r->generated && r->n > 0) {
            GenDesc &g = gen[P.gen++];
            g.k = r->k;
            g.v = r->with_values ? r->v : nullptr;
            g.n = static_cast<uint32_t>(r->n);
            g.first_chunk = P.gen_chunks;
            P.gen_chunks += static_cast<uint32_t>((r->n + kGenChunk - 1) / kGenChunk);
            memset(&g.g, 0, sizeof g.g);
            g.g.dist = r->gen.dist;
            g.g.state = r->gen.state;
            memcpy(g.g.dictionary, r->gen.dictionary, sizeof g.g.dictionary);
            memcpy(g.g.thresholds, r->gen.thresholds, sizeof g.g.thresholds);
        }
        if (r->n < 2) continue;  // nothing to sort
        if (it.small) {
            int c = static_cast<int>(s->classes.count) - 1;
            for (int q = c; q >= 0; --q)
                if (r->n <= s->classes.cls[q].max_n) c = q;
            lists[static_cast<size_t>(c) * stride + hp->count[c]++] = static_cast<uint32_t>(i);
            ++P.small[c];
        } else {
            lists[static_cast<size_t>(kSegLarge) * stride + hp->count[kSegLarge]++] = static_cast<uint32_t>(i);
            ++P.tiled;
            P.tiles += (r->n + kSegTile - 1) / kSegTile;
            if (it.fresh) {
                hlist[hh->count[kSegLarge]++] = static_cast<uint32_t>(i);
                ++P.fresh_tiled;
            }
        }
    }
    return P;
}

// Enqueues a built step on the server's stream and records its event.
rt_status enqueue_step(rt_server *s, StepSlot &slot, const StepPlan &P) {
    const Meta &m = s->meta;
    hipStream_t st = s->stream;
    const uint32_t stride = s->max_active;
    char *dm = s->dmeta;
    char *hb = slot.host;
    if (P.tiles > m.max_tiles) return set_error(RT_ERR_HIP, "server: step of %zu tiles exceeds %u", P.tiles, m.max_tiles);
    hipError_t e = hipMemcpyAsync(dm, hb, m.block_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && P.gen)
        e = hipMemcpyAsync(dm + m.gen, hb + m.block_bytes, sizeof(GenDesc) * P.gen, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "server: step upload: %s", hipGetErrorString(e));

    SegHeader *d_hp = reinterpret_cast<SegHeader *>(dm + m.hdr_pass);
    SegHeader *d_hh = reinterpret_cast<SegHeader *>(dm + m.hdr_hist);
    const SegDesc *d_descs = reinterpret_cast<const SegDesc *>(dm + m.descs);
    uint32_t *d_lists = reinterpret_cast<uint32_t *>(dm + m.lists_pass);
    uint32_t *d_hlist = reinterpret_cast<uint32_t *>(dm + m.list_hist) + static_cast<size_t>(kSegLarge) * stride;
    uint32_t *d_plist = d_lists + static_cast<size_t>(kSegLarge) * stride;
    uint32_t *d_first_p = reinterpret_cast<uint32_t *>(dm + m.first_pass);
    uint32_t *d_first_h = reinterpret_cast<uint32_t *>(dm + m.first_hist);
    SegDesc *d_seg_p = reinterpret_cast<SegDesc *>(dm + m.seg_pass);
    SegDesc *d_seg_h = reinterpret_cast<SegDesc *>(dm + m.seg_hist);
    uint32_t *d_hist = reinterpret_cast<uint32_t *>(dm + m.hist);
    uint32_t *d_base = reinterpret_cast<uint32_t *>(dm + m.base);
    uint32_t *d_status = reinterpret_cast<uint32_t *>(dm + m.status);
    const uint32_t cus = static_cast<uint32_t>(device_cu_count());
    auto grid = [](size_t want, uint32_t cap) {
        return static_cast<uint32_t>(std::max<size_t>(1, std::min<size_t>(want, cap)));
    };

    for (const auto &c : P.copies) {  // out-of-place inputs into their outputs
        e = hipMemcpyAsync(std::get<0>(c), std::get<1>(c), std::get<2>(c), hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return set_error(RT_ERR_HIP, "server: input copy: %s", hipGetErrorString(e));
    }
    if (P.gen)  // inputs of the fresh generated requests
        hipLaunchKernelGGL(k_srv_generate, dim3(P.gen_chunks), dim3(256), 0, st,
                           reinterpret_cast<const GenDesc *>(dm + m.gen), P.gen);
    if (P.fresh_tiled) {  // histograms and prefix sums of fresh tiled requests
        hipLaunchKernelGGL(k_srv_clear_rows, dim3(grid(P.fresh_tiled, cus * 4)), dim3(256), 0, st, d_descs, d_hlist,
                           d_hh, d_hist);
        hipLaunchKernelGGL(k_seg_tiles, dim3(1), dim3(1024), 0, st, d_descs, d_hlist, d_first_h, d_hh, stride,
                           m.max_tiles, static_cast<uint32_t>(kSegTile));
        hipLaunchKernelGGL(k_seg_tilemap, dim3(grid((P.tiles + 255) / 256, cus * 4)), dim3(256), 0, st, d_descs,
                           d_hlist, d_first_h, d_hh, d_seg_h, 1u);
        hipLaunchKernelGGL((k_seg_histogram<512, 16>), dim3(grid(P.tiles, cus * 2)), dim3(512), 0, st, d_seg_h,
                           d_hh, d_hist, static_cast<uint32_t>(kSegTile),
                           (1u << kSegPasses) - 1u);
        hipLaunchKernelGGL(k_seg_plan, dim3(grid(P.fresh_tiled, cus * 4)), dim3(256), 0, st, d_descs, d_hlist, d_hh,
                           d_hist, d_base);
    }
    if (P.tiled) {  // one pass of every tiled request, each at its own pass
        hipLaunchKernelGGL(k_fill_zero, dim3(grid((P.tiles * kSegRadix + 4095) / 4096, 4096)), dim3(256), 0, st,
                           d_status, P.tiles * kSegRadix);
        hipLaunchKernelGGL(k_seg_tiles, dim3(1), dim3(1024), 0, st, d_descs, d_plist, d_first_p, d_hp, stride,
                           m.max_tiles, static_cast<uint32_t>(kSegTile));
        // XCD chunks when the step's tiled requests are long (see seg_chunk_count)
        const uint32_t nchunks = seg_chunk_count(P.tiles * kSegTile, P.tiled, kSegTile);
        hipLaunchKernelGGL(k_seg_tilemap, dim3(grid((P.tiles + 255) / 256, cus * 4)), dim3(256), 0, st, d_descs,
                           d_plist, d_first_p, d_hp, d_seg_p, nchunks);
        uint32_t *ctr = reinterpret_cast<uint32_t *>(d_hp) + offsetof(SegHeader, chunk_ctr) / 4;
        uint32_t *err = reinterpret_cast<uint32_t *>(d_hp) + offsetof(SegHeader, error) / 4;
        // a server holds one value layout (checked at submit), so one
        // kernel flavour serves every request of the step
        if (P.vals)
            hipLaunchKernelGGL((k_seg_onesweep<1024, 16, true, uint32_t>), dim3(static_cast<uint32_t>(P.tiles)),
                               dim3(1024), 0, st, d_seg_p, d_hp, -1, d_base, d_status,
                               ctr, err, nchunks, 0u);
        else
            hipLaunchKernelGGL((k_seg_onesweep<1024, 16, false, uint32_t>), dim3(static_cast<uint32_t>(P.tiles)),
                               dim3(1024), 0, st, d_seg_p, d_hp, -1, d_base, d_status,
                               ctr, err, nchunks, 0u);
    }
    for (uint32_t c = 0; c < s->classes.count; ++c)  // small requests, whole in LDS
        if (P.small[c])
            launch_seg_small(s->classes.cls[c], P.vals, P.small[c], st, d_descs,
                             d_lists + static_cast<size_t>(c) * stride, d_hp, static_cast<int>(c), 32, 0);
    e = hipGetLastError();
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "server: launch: %s", hipGetErrorString(e));
    // the error words of both headers come back with the step
    char *rb = hb + m.block_bytes + sizeof(GenDesc) * s->max_active;
    e = hipMemcpyAsync(rb, dm + m.hdr_pass, 2 * 256, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(slot.done, st);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "server: step: %s", hipGetErrorString(e));
    return RT_OK;
}

// Retires the oldest step in flight once its event has fired (waiting for
// it when `block`): the scheduler completes it, with the failure of the
// step if its enqueue, the device or a lookback word reported one.  Returns
// whether a step was retired.
bool retire_oldest(rt_server *s, bool block) {
    if (s->ring_count == 0) return false;
    StepSlot &slot = s->ring[s->ring_head];
    hipError_t e = block ? hipEventSynchronize(slot.done) : hipEventQuery(slot.done);
    if (e == hipErrorNotReady) return false;
    const char *rb = slot.host + s->meta.block_bytes + sizeof(GenDesc) * s->max_active;
    rt_status status = slot.enqueue_status;
    std::string why = slot.enqueue_error;
    if (status == RT_OK && e != hipSuccess) {
        status = RT_ERR_HIP;
        why = std::string("server: step failed: ") + hipGetErrorString(e);
    } else if (status == RT_OK) {
        const uint32_t err =
            reinterpret_cast<const SegHeader *>(rb)->error | reinterpret_cast<const SegHeader *>(rb + 256)->error;
        if (err) {
            status = RT_ERR_HIP;
            char buf[96];
            snprintf(buf, sizeof buf, "server: device error word 0x%x", err);
            why = buf;
        }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->sched->complete(slot.step, status, why, now_us());
    s->ring_head = (s->ring_head + 1) % kRing;
    --s->ring_count;
    s->cv_done.notify_all();
    return true;
}

void scheduler(rt_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<Request *> admitted;
    for (;;) {
        while (retire_oldest(s, false)) {
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) break;
        if (s->ring_count >= s->depth) {  // enough steps in flight: wait for the oldest
            lk.unlock();
            retire_oldest(s, true);
            continue;
        }
        admitted.clear();
        s->sched->admit(&admitted);
        place(s, admitted);
        if (!s->sched->has_active()) {
            if (s->ring_count) {
                lk.unlock();
                retire_oldest(s, true);
                continue;
            }
            // idle, or the head of the queue waits for memory to be released
            if (!s->sched->has_queued())
                s->cv_work.wait(lk, [&] { return s->stop || s->sched->has_queued() || s->sched->has_active(); });
            else
                s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
            continue;
        }
        StepSlot &slot = s->ring[(s->ring_head + s->ring_count) % kRing];
        const StepPlan P = build_step(s, slot);
        ++s->ring_count;
        lk.unlock();
        const rt_status st = enqueue_step(s, slot, P);
        if (st != RT_OK) {
            // part of this step may have been enqueued: let the stream drain,
            // then retire it as failed (its requests end or leave; the
            // others are untouched)
            (void)hipStreamSynchronize(s->stream);
            slot.enqueue_status = st;
            slot.enqueue_error = last_error();
            (void)hipEventRecord(slot.done, s->stream);
        }
    }
    // drain: finish what is in flight, so waiters see their results
    while (s->ring_count) retire_oldest(s, true);
}

rt_status enqueue(rt_server *s, std::unique_ptr<Request> r, uint64_t *ticket) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return set_error(RT_ERR_CANCELLED, "server: stopping");
    // one value layout per server (the step kernels are instantiated for it)
    const int held = s->sched->held_layout();
    if (held >= 0 && held != (r->with_values ? 1 : 0))
        return set_error(RT_ERR_INVALID_ARG, "server: mixing keys-only and key/value requests is not supported");
    *ticket = s->sched->submit(std::move(r), now_us());
    s->cv_work.notify_one();
    return RT_OK;
}

}  // namespace

extern "C" rt_status rt_server_create(size_t hbm_budget_bytes, uint32_t max_active, rt_server **out) {
    if (out == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_create: out is NULL");
    *out = nullptr;
    if (max_active == 0 || max_active > (1u << 20))
        return set_error(RT_ERR_INVALID_ARG, "rt_server_create: max_active %u outside 1..2^20", max_active);
    if (hbm_budget_bytes < (1u << 20))
        return set_error(RT_ERR_INVALID_ARG, "rt_server_create: budget below 1 MiB");
    std::unique_ptr<rt_server> s(new rt_server());
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "rt_server_create: %s", hipGetErrorString(e));
    s->arena_bytes = round_up(hbm_budget_bytes);
    s->max_active = max_active;
    s->classes = rt::seg_class_table();
    s->meta = make_meta(max_active, s->arena_bytes, s->classes.lds_max());
    e = hipMalloc(reinterpret_cast<void **>(&s->arena), s->arena_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RT_ERR_OUT_OF_MEMORY, "rt_server_create: arena of %zu bytes: %s", s->arena_bytes,
                         hipGetErrorString(e));
    }
    e = hipMalloc(reinterpret_cast<void **>(&s->dmeta), s->meta.total);
    for (int i = 0; i < kRing && e == hipSuccess; ++i) {
        e = hipHostMalloc(reinterpret_cast<void **>(&s->ring[i].host), slot_bytes(s->meta, max_active));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ring[i].done, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->io, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        if (s->dmeta) (void)hipFree(s->dmeta);
        for (int i = 0; i < kRing; ++i) {
            if (s->ring[i].host) (void)hipHostFree(s->ring[i].host);
            if (s->ring[i].done) (void)hipEventDestroy(s->ring[i].done);
        }
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->io) (void)hipStreamDestroy(s->io);
        (void)hipFree(s->arena);
        return set_error(RT_ERR_OUT_OF_MEMORY, "rt_server_create: metadata: %s", hipGetErrorString(e));
    }
    if (const char *d = getenv("RT_SERVER_DEPTH")) {  // steps in flight (tuning knob)
        const int v = atoi(d);
        if (v >= 1 && v <= kRing) s->depth = v;
    }
    s->sched.reset(new sched::Scheduler(s->arena_bytes, max_active, s->classes.lds_max(), kSegPasses));
    rt_server *raw = s.release();
    raw->thr = std::thread(scheduler, raw);
    *out = raw;
    return RT_OK;
}

static rt_status check_request_size(rt_server *s, size_t n, bool generated, bool with_values, const char *what) {
    if (n > kMaxRequestItems) return set_error(RT_ERR_TOO_LARGE, "%s: n = %zu, the server limit is 2^30 - 1", what, n);
    const size_t need = s->sched->footprint(n, generated, with_values);
    if (need > s->arena_bytes)
        return set_error(RT_ERR_BUDGET, "%s: %zu bytes needed, the budget is %zu", what, need, s->arena_bytes);
    return RT_OK;
}

// Whether two u32 arrays of n items share any byte.
static bool overlap(const void *a, const void *b, size_t n) {
    if (a == nullptr || b == nullptr || n == 0) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    const uintptr_t bytes = n * sizeof(uint32_t);
    return x < y + bytes && y < x + bytes;
}

extern "C" rt_status rt_server_submit(rt_server *s, const uint32_t *keys, const uint32_t *vals, uint32_t *out_keys,
                                      uint32_t *out_vals, size_t n, uint64_t *ticket) {
    if (s == nullptr || ticket == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: NULL argument");
    if (n > 0 && keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: keys is NULL");
    // no output arrays (or the inputs themselves): sorted in place
    const bool in_place = out_keys == nullptr || out_keys == keys;
    if (in_place && out_vals != nullptr && out_vals != vals)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: out_vals given for an in-place request");
    if (!in_place && vals != nullptr && out_vals == nullptr)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: out_vals is NULL for an out-of-place request");
    uint32_t *k = in_place ? const_cast<uint32_t *>(keys) : out_keys;
    uint32_t *v = vals == nullptr ? nullptr : (in_place ? const_cast<uint32_t *>(vals) : out_vals);
    if ((reinterpret_cast<uintptr_t>(keys) | reinterpret_cast<uintptr_t>(vals) | reinterpret_cast<uintptr_t>(k) |
         reinterpret_cast<uintptr_t>(v)) & 3u)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: arrays must be 4-byte aligned");
    if (overlap(k, v, n)) return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: keys and values overlap");
    if (!in_place && (overlap(keys, k, n) || overlap(keys, v, n) || overlap(vals, k, n) || overlap(vals, v, n)))
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit: inputs and outputs overlap");
    rt_status st = check_request_size(s, n, false, vals != nullptr, "rt_server_submit");
    if (st != RT_OK) return st;
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->k = k;
    r->v = v;
    if (!in_place) {
        r->in_k = keys;
        r->in_v = vals;
    }
    r->with_values = vals != nullptr;
    return enqueue(s, std::move(r), ticket);
}

extern "C" rt_status rt_server_submit_generated(rt_server *s, const rt_gen_params *params, size_t n,
                                                uint64_t *ticket) {
    if (s == nullptr || params == nullptr || ticket == nullptr)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit_generated: NULL argument");
    if (params->dist > RT_DIST_ZIPF16)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_submit_generated: unknown dist %u", params->dist);
    rt_status st = check_request_size(s, n, true, true, "rt_server_submit_generated");
    if (st != RT_OK) return st;
    std::unique_ptr<Request> r(new Request());
    r->n = n;
    r->generated = true;
    r->with_values = true;
    r->gen = *params;
    return enqueue(s, std::move(r), ticket);
}

// Reports a finished request (mu held): its latency and status; a request
// with nothing left to fetch is dropped.
static rt_status collect(rt_server *s, uint64_t ticket, double *latency_us, const char *what) {
    std::string why;
    const rt_status st = s->sched->collect(ticket, latency_us, &why);
    if (st == RT_ERR_NOT_FOUND)
        return set_error(st, "%s: request %llu was collected by another wait", what, (unsigned long long)ticket);
    if (st != RT_OK)
        return set_error(st, "%s: request %llu failed: %s", what, (unsigned long long)ticket, why.c_str());
    return RT_OK;
}

extern "C" rt_status rt_server_wait(rt_server *s, uint64_t ticket, int64_t timeout_us, double *latency_us) {
    if (s == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_wait: server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const Request *r = s->sched->find(ticket);
    if (r == nullptr || r->collected)
        return set_error(RT_ERR_NOT_FOUND, "rt_server_wait: no request %llu", (unsigned long long)ticket);
    // looked up afresh on every wake-up: another waiter on the same ticket
    // may have taken it meanwhile
    auto done = [&] { return s->sched->done(ticket); };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return set_error(RT_ERR_TIMEOUT, "rt_server_wait: request %llu still running", (unsigned long long)ticket);
    }
    return collect(s, ticket, latency_us, "rt_server_wait");
}

extern "C" rt_status rt_server_wait_any(rt_server *s, int64_t timeout_us, uint64_t *ticket, double *latency_us) {
    if (s == nullptr || ticket == nullptr)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_wait_any: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] { return s->sched->next_finished() != 0; };
    if (!ready()) {
        if (s->sched->uncollected() == 0)
            return set_error(RT_ERR_NOT_FOUND, "rt_server_wait_any: no request outstanding");
        if (timeout_us < 0) {
            s->cv_done.wait(lk, ready);
        } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
            return set_error(RT_ERR_TIMEOUT, "rt_server_wait_any: nothing finished");
        }
    }
    *ticket = s->sched->next_finished();
    return collect(s, *ticket, latency_us, "rt_server_wait_any");
}

extern "C" rt_status rt_server_cancel(rt_server *s, uint64_t ticket) {
    if (s == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_cancel: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    const rt_status st = s->sched->cancel(ticket, now_us());
    if (st == RT_ERR_NOT_FOUND)
        return set_error(st, "rt_server_cancel: no request %llu", (unsigned long long)ticket);
    if (st == RT_ERR_INVALID_ARG)
        return set_error(st, "rt_server_cancel: request %llu has finished or its last pass is under way",
                         (unsigned long long)ticket);
    s->cv_done.notify_all();  // a queued request has ended
    s->cv_work.notify_one();  // an admitted one leaves at the next step
    return RT_OK;
}

extern "C" rt_status rt_server_fetch(rt_server *s, uint64_t ticket, uint32_t *out_keys, uint32_t *out_vals) {
    if (s == nullptr || out_keys == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_fetch: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    const Request *r = s->sched->find(ticket);
    if (r == nullptr || !r->generated)
        return set_error(RT_ERR_NOT_FOUND, "rt_server_fetch: no generated request %llu", (unsigned long long)ticket);
    if (r->state != sched::kDone)
        return set_error(RT_ERR_INVALID_ARG, "rt_server_fetch: request %llu not finished", (unsigned long long)ticket);
    if (r->status != RT_OK) return set_error(r->status, "rt_server_fetch: request %llu failed", (unsigned long long)ticket);
    const size_t bytes = r->n * sizeof(uint32_t);
    hipError_t e = hipSuccess;
    if (bytes) {
        e = hipMemcpyAsync(out_keys, r->k, bytes, hipMemcpyDeviceToDevice, s->io);
        if (e == hipSuccess && out_vals) e = hipMemcpyAsync(out_vals, r->v, bytes, hipMemcpyDeviceToDevice, s->io);
        if (e == hipSuccess) e = hipStreamSynchronize(s->io);
    }
    if (e != hipSuccess) return set_error(RT_ERR_HIP, "rt_server_fetch: %s", hipGetErrorString(e));
    (void)s->sched->release(ticket);
    s->cv_work.notify_one();  // memory came free
    return RT_OK;
}

extern "C" rt_status rt_server_release(rt_server *s, uint64_t ticket) {
    if (s == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_release: server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    const rt_status st = s->sched->release(ticket);
    if (st == RT_ERR_NOT_FOUND)
        return set_error(st, "rt_server_release: no request %llu", (unsigned long long)ticket);
    if (st != RT_OK)
        return set_error(st, "rt_server_release: request %llu not finished", (unsigned long long)ticket);
    s->cv_work.notify_one();  // memory came free
    return RT_OK;
}

extern "C" rt_status rt_server_stats_ex(rt_server *s, double *p50_us, double *p99_us, double *gkeys_per_s,
                                        uint64_t *completed, size_t *peak_bytes) {
    if (s == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_server_stats: server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    double per_us = 0;
    s->sched->stats(p50_us, p99_us, &per_us, completed);
    if (gkeys_per_s) *gkeys_per_s = per_us / 1e3;
    if (peak_bytes) *peak_bytes = s->sched->peak();
    return RT_OK;
}

extern "C" rt_status rt_server_stats(rt_server *s, double *p50_us, double *p99_us, double *gkeys_per_s) {
    return rt_server_stats_ex(s, p50_us, p99_us, gkeys_per_s, nullptr, nullptr);
}

extern "C" rt_status rt_server_replay(rt_server *s, const rt_replay_request *reqs, size_t count, double *latency_us,
                                     double *span_us) {
    if (s == nullptr || (count > 0 && (reqs == nullptr || latency_us == nullptr)))
        return set_error(RT_ERR_INVALID_ARG, "rt_server_replay: NULL argument");
    for (size_t i = 0; i < count; ++i) {
        latency_us[i] = -1.0;
        if (i && reqs[i].arrival_us < reqs[i - 1].arrival_us)
            return set_error(RT_ERR_INVALID_ARG, "rt_server_replay: arrivals decrease at request %zu", i);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->sched->uncollected())
            return set_error(RT_ERR_INVALID_ARG, "rt_server_replay: requests are outstanding");
    }
    if (span_us) *span_us = 0.0;
    if (count == 0) return RT_OK;

    std::mutex mu;  // ticket -> request index, and the submitter's outcome
    std::unordered_map<uint64_t, size_t> index_of;
    size_t submitted = 0;
    bool submit_done = false;
    rt_status submit_status = RT_OK;
    std::string submit_error;
    const double t0 = now_us() + 1000.0;  // the trace starts 1 ms from now

    std::thread submitter([&] {
        for (size_t i = 0; i < count; ++i) {
            const double at = t0 + reqs[i].arrival_us;
            for (double now = now_us(); now < at; now = now_us())
                if (at - now > 300.0) std::this_thread::sleep_for(std::chrono::microseconds(static_cast<int64_t>(at - now - 200.0)));
            uint64_t ticket = 0;
            const rt_status st = rt_server_submit_generated(s, &reqs[i].params, static_cast<size_t>(reqs[i].n), &ticket);
            std::lock_guard<std::mutex> g(mu);
            if (st != RT_OK) {
                submit_status = st;
                submit_error = last_error();
                break;
            }
            index_of[ticket] = i;
            submitted = i + 1;
        }
        std::lock_guard<std::mutex> g(mu);
        submit_done = true;
    });

    rt_status result = RT_OK;
    std::string result_error;
    size_t collected = 0;
    double last_done = t0;
    for (;;) {
        {
            std::lock_guard<std::mutex> g(mu);
            if (submit_done && collected == submitted) break;
        }
        uint64_t ticket = 0;
        double ignored = 0;
        const rt_status st = rt_server_wait_any(s, 20000, &ticket, &ignored);
        if (st == RT_ERR_TIMEOUT) continue;  // nothing finished yet
        if (st == RT_ERR_NOT_FOUND) {        // all collected, the next arrival still ahead:
            std::this_thread::sleep_for(std::chrono::microseconds(20));  // leave the lock to the scheduler
            continue;
        }
        // the request may finish before the submitter has recorded its
        // ticket: look until it is there or the submitter has stopped
        size_t i = count;
        for (bool stopped = false; i == count && !stopped;) {
            std::lock_guard<std::mutex> g(mu);
            auto f = index_of.find(ticket);
            if (f != index_of.end()) i = f->second;
            stopped = submit_done;
        }
        if (i == count) {  // not from this trace (another client broke the rule)
            (void)rt_server_release(s, ticket);
            continue;
        }
        if (st == RT_OK) {
            double done = 0;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (const Request *r = s->sched->find(ticket)) done = r->t_done;
            }
            latency_us[i] = done - (t0 + reqs[i].arrival_us);
            last_done = std::max(last_done, done);
        } else if (result == RT_OK) {
            result = st;
            result_error = last_error();
        }
        (void)rt_server_release(s, ticket);
        ++collected;
    }
    submitter.join();
    if (span_us) *span_us = last_done - t0;
    if (submit_status != RT_OK)
        return set_error(submit_status, "rt_server_replay: submission %zu refused: %s", submitted,
                         submit_error.c_str());
    if (result != RT_OK) return set_error(result, "rt_server_replay: %s", result_error.c_str());
    return RT_OK;
}

extern "C" rt_status rt_server_destroy(rt_server *s) {
    if (s == nullptr) return RT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->thr.joinable()) s->thr.join();
    (void)hipStreamSynchronize(s->stream);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->sched->cancel_all(now_us());
        s->cv_done.notify_all();
    }
    for (int i = 0; i < kRing; ++i) {
        (void)hipEventDestroy(s->ring[i].done);
        (void)hipHostFree(s->ring[i].host);
    }
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->io);
    (void)hipFree(s->dmeta);
    (void)hipFree(s->arena);
    delete s;
    return RT_OK;
}
