// Request server (edt_serve_*): continuous batching of independent images.
//
// Submitters append requests to a FIFO queue.  One scheduler thread per
// server loops over three steps:
//   1. retire: every launched group whose completion event has fired gives
//      back its arena blocks and launch slot, and its requests are marked
//      done (latency = now - submission time);
//   2. admit and launch: while a launch slot is free, the longest prefix of
//      the queue whose workspaces fit in the arena (at most max_group
//      requests) becomes one group and is launched on the next stream, after
//      the events that mark each request's mask as ready; a group of two or
//      more runs as one batch over a table staged through pinned memory, a
//      lone request (or one wider than the one-lane-per-row pass takes,
//      which is always launched alone) as a single transform;
//   3. wait: spin (yielding) while work is in flight, sleep while idle.
// Requests that arrive while groups run are picked up by the next launch, so
// the batch size follows the load.  Admission is strictly in arrival order: a
// request that does not fit waits for memory to come back, and so does every
// request behind it, which bounds every request's wait.
#include "../../include/edt.h"
#include "edt_internal.h"
#include "serve_core.h"

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;
constexpr int32_t kPending = edt::TicketBook::kPending;  // request state before completion
static_assert(EDT_OK == 0 && kPending != EDT_OK, "the ticket book takes 0 for success");

struct Req {
    uint64_t ticket;
    edt_request r;
    size_t bytes;      // workspace
    size_t off;        // arena offset once admitted
    hipEvent_t ready;  // recorded on the caller's stream at submission
    Clock::time_point t0;
};

struct Group {
    std::vector<Req> reqs;
    int slot = -1;  // launch slot: pinned staging + device table
    int stream = 0;
    hipEvent_t done = nullptr;
    bool failed = false;
};

}  // namespace

struct edt_server {
    edt_serve_config cfg{};
    int device = 0;
    uint8_t* tables = nullptr;  // start of the arena: one launch table per slot
    uint8_t* arena = nullptr;   // the rest: request workspaces
    size_t table_len = 0;       // bytes of one launch table (max_group images)

    // scheduler-private
    edt::Arena alloc;
    std::vector<Group> inflight;
    std::vector<int> free_slots;
    std::vector<uint8_t*> staging;  // pinned host, one per slot
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    bool broken = false;

    // shared with submitters (under mu)
    std::mutex mu;
    std::condition_variable wake;     // the scheduler
    std::condition_variable done_cv;  // waiters
    std::deque<Req> queue;
    std::vector<hipEvent_t> events;   // idle events
    edt::TicketBook book;             // per-ticket status, latencies
    size_t live = 0;                  // queued or running requests
    bool stop = false;
    bool any = false;
    Clock::time_point t_first, t_last;
    edt_serve_counters st{};

    std::thread th;
};

namespace {

hipEvent_t take_event(edt_server* s) {  // under mu
    if (!s->events.empty()) {
        hipEvent_t e = s->events.back();
        s->events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Move requests from the head of the queue into g while they fit.
void form_group(edt_server* s, Group& g) {
    std::lock_guard<std::mutex> lk(s->mu);
    const int cap = s->cfg.max_group;
    while (!s->queue.empty() && (int)g.reqs.size() < cap) {
        Req& r = s->queue.front();
        // images whose rows the one-lane-per-row pass does not take have
        // enough rows of work to fill the GPU alone, and the single-image row
        // pass is the faster one for them: they are launched alone
        const bool wide = r.r.W > edt::kLaneMaxW;
        if (wide && !g.reqs.empty()) break;
        size_t off = 0;
        if (!s->alloc.alloc(r.bytes, &off)) break;
        r.off = off;
        g.reqs.push_back(r);
        s->queue.pop_front();
        if (wide) break;
    }
}

edt::Img image_of(const edt_server* s, const Req& q) {
    edt::Img g;
    g.mask = q.r.mask;
    g.mpitch = q.r.mask_pitch;
    g.dist = q.r.dist_sq;
    g.feat = q.r.feature;
    g.opitch = q.r.out_pitch;
    g.ws = s->arena + q.off;
    g.H = q.r.H;
    g.W = q.r.W;
    g.pol = q.r.polarity;
    g.metric = EDT_METRIC_EUCLIDEAN_SQ;
    return g;
}

// Enqueue a group; false if a HIP call failed (the group is then failed).
bool launch(edt_server* s, Group& g) {
    if (s->broken) return false;
    const hipStream_t st = s->streams[g.stream];
    for (const Req& q : g.reqs)
        if (hipStreamWaitEvent(st, q.ready, 0) != hipSuccess) return false;
    const int n = (int)g.reqs.size();
    if (n == 1) return edt::enqueue_single(image_of(s, g.reqs[0]), st) == hipSuccess;
    std::vector<edt::BatchImage> img(n);
    for (int k = 0; k < n; ++k) {
        const Req& q = g.reqs[k];
        edt::BatchImage& b = img[k];
        b.mask_off = (int64_t)reinterpret_cast<uintptr_t>(q.r.mask);
        b.mpitch = q.r.mask_pitch;
        b.dist_off = (int64_t)(reinterpret_cast<uintptr_t>(q.r.dist_sq) / 4);
        b.feat_off = (int64_t)(reinterpret_cast<uintptr_t>(q.r.feature) / 4);
        b.opitch = q.r.out_pitch;
        b.ws_off = (int64_t)q.off;
        b.H = q.r.H;
        b.W = q.r.W;
        b.pol = q.r.polarity;
        b.outs = (q.r.dist_sq ? edt::kOutDist : 0) | (q.r.feature ? edt::kOutFeat : 0);
        b.tr = 0;
        b.pad_ = 0;
    }
    int totals[edt::kPhases], max_w = 0;
    uint8_t* host = s->staging[g.slot];
    if (edt::pack_table(img.data(), n, edt::kLaneMaxW, host, totals, &max_w) != EDT_OK)
        return false;
    uint8_t* dev = s->tables + (size_t)g.slot * s->table_len;
    if (hipMemcpyAsync(dev, host, edt::table_bytes(n), hipMemcpyHostToDevice, st) != hipSuccess)
        return false;
    edt::BatchTable t = edt::table_view(dev, n, totals);
    t.ws_base = reinterpret_cast<uintptr_t>(s->arena);
    return edt::enqueue_batch(t, totals, max_w, st) == hipSuccess;
}

// Give back what a finished group holds and publish its requests' status.
void finish(edt_server* s, Group& g, int32_t status) {
    for (const Req& q : g.reqs) s->alloc.release(q.off, q.bytes);
    s->free_slots.push_back(g.slot);
    const Clock::time_point now = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (const Req& q : g.reqs) {
            s->book.complete(q.ticket, status,
                             std::chrono::duration<double, std::nano>(now - q.t0).count());
            s->st.done += 1;
            if (status != EDT_OK)
                s->st.failed += 1;
            else
                s->st.pixels_done += (uint64_t)q.r.H * (uint64_t)q.r.W;
            s->events.push_back(q.ready);
            s->live -= 1;
        }
        if (g.done) s->events.push_back(g.done);
        s->t_last = now;
        s->st.hbm_in_use = s->alloc.in_use();
    }
    s->done_cv.notify_all();
}

void scheduler(edt_server* s) {
    if (hipSetDevice(s->device) != hipSuccess) s->broken = true;
    for (;;) {
        // 1. retire
        for (size_t k = 0; k < s->inflight.size();) {
            Group& g = s->inflight[k];
            hipError_t q = hipSuccess;
            if (!g.failed) q = hipEventQuery(g.done);
            if (q == hipErrorNotReady) {
                ++k;
                continue;
            }
            if (g.failed) (void)hipStreamSynchronize(s->streams[g.stream]);
            finish(s, g, (g.failed || q != hipSuccess) ? EDT_ERR_DEVICE : EDT_OK);
            s->inflight[k] = std::move(s->inflight.back());
            s->inflight.pop_back();
        }
        // 2. admit and launch
        while (!s->free_slots.empty()) {
            Group g;
            form_group(s, g);
            if (g.reqs.empty()) break;
            g.slot = s->free_slots.back();
            s->free_slots.pop_back();
            g.stream = s->next_stream;
            s->next_stream = (s->next_stream + 1) % (int)s->streams.size();
            {
                std::lock_guard<std::mutex> lk(s->mu);
                g.done = take_event(s);
                s->st.launches += 1;
                s->st.hbm_in_use = s->alloc.in_use();
                s->st.hbm_high_water = s->alloc.high_water();
            }
            g.failed = g.done == nullptr || !launch(s, g) ||
                       hipEventRecord(g.done, s->streams[g.stream]) != hipSuccess;
            s->inflight.push_back(std::move(g));
        }
        // 3. wait
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && s->queue.empty() && s->inflight.empty()) break;
        if (s->inflight.empty()) {
            s->wake.wait(lk, [s] { return s->stop || !s->queue.empty(); });
        } else {
            lk.unlock();
            std::this_thread::yield();
        }
    }
}

void destroy_parts(edt_server* s) {
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    s->events.clear();
    for (uint8_t* p : s->staging)
        if (p) (void)hipHostFree(p);
    s->staging.clear();
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    s->streams.clear();
}

}  // namespace

extern "C" {

size_t edt_serve_reserved_bytes(const edt_serve_config* cfg) {
    if (!cfg || cfg->n_streams < 1 || cfg->n_streams > EDT_SERVE_MAX_STREAMS ||
        cfg->max_group < 0 || cfg->max_group > EDT_SERVE_MAX_GROUP)
        return 0;
    const int group = cfg->max_group == 0 ? EDT_SERVE_MAX_GROUP : cfg->max_group;
    return (size_t)(2 * cfg->n_streams) * edt::Arena::round(edt::table_bytes(group));
}

edt_status edt_serve_create(const edt_serve_config* cfg, void* arena, size_t arena_bytes,
                            edt_server** out) {
    if (!cfg || !arena || !out) return EDT_ERR_INVALID_ARG;
    *out = nullptr;
    if ((reinterpret_cast<uintptr_t>(arena) & 255) != 0) return EDT_ERR_INVALID_ARG;
    if (cfg->max_inflight < 1 || cfg->n_streams < 1 || cfg->n_streams > EDT_SERVE_MAX_STREAMS ||
        cfg->max_group < 0 || cfg->max_group > EDT_SERVE_MAX_GROUP)
        return EDT_ERR_INVALID_ARG;
    size_t budget = cfg->hbm_budget_bytes == 0 ? arena_bytes : cfg->hbm_budget_bytes;
    if (budget > arena_bytes) return EDT_ERR_INVALID_ARG;
    budget = budget / edt::Arena::kAlign * edt::Arena::kAlign;

    edt_server* s = new (std::nothrow) edt_server;
    if (!s) return EDT_ERR_OUT_OF_MEMORY;
    s->cfg = *cfg;
    if (s->cfg.max_group == 0) s->cfg.max_group = EDT_SERVE_MAX_GROUP;
    s->table_len = edt::Arena::round(edt::table_bytes(s->cfg.max_group));
    const int slots = 2 * s->cfg.n_streams;
    // the launch tables come first in the arena and out of the budget
    const size_t reserved = edt_serve_reserved_bytes(cfg);
    if (budget <= reserved) {
        delete s;
        return EDT_ERR_INVALID_ARG;
    }
    s->tables = static_cast<uint8_t*>(arena);
    s->arena = s->tables + reserved;
    s->alloc.reset(budget - reserved);
    bool ok = hipGetDevice(&s->device) == hipSuccess;
    for (int k = 0; k < s->cfg.n_streams && ok; ++k) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
    }
    for (int k = 0; k < slots && ok; ++k) {
        void* p = nullptr;
        ok = hipHostMalloc(&p, s->table_len, hipHostMallocDefault) == hipSuccess;
        if (ok) {
            s->staging.push_back(static_cast<uint8_t*>(p));
            s->free_slots.push_back(k);
        }
    }
    if (!ok) {
        destroy_parts(s);
        delete s;
        return EDT_ERR_DEVICE;
    }
    try {
        s->th = std::thread(scheduler, s);
    } catch (...) {
        destroy_parts(s);
        delete s;
        return EDT_ERR_OUT_OF_MEMORY;
    }
    *out = s;
    return EDT_OK;
}

edt_status edt_serve_submit(edt_server* s, const edt_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket) return EDT_ERR_INVALID_ARG;
    const int64_t opitch = r->out_pitch;
    edt_status c = edt::check_image(r->mask, r->H, r->W, r->mask_pitch, r->polarity,
                                    EDT_METRIC_EUCLIDEAN_SQ, opitch);
    if (c == EDT_OK && (r->reserved != 0 || (!r->dist_sq && !r->feature))) c = EDT_ERR_INVALID_ARG;
    if (c == EDT_OK && ((reinterpret_cast<uintptr_t>(r->dist_sq) & 3) != 0 ||
                        (reinterpret_cast<uintptr_t>(r->feature) & 3) != 0))
        c = EDT_ERR_INVALID_ARG;
    // a request that may share a launch may take the one-lane-per-row pass,
    // whose envelopes its workspace then holds as well
    const bool stack = s->cfg.max_group > 1 && edt::lane_image(r->H, r->W);
    const size_t bytes = c == EDT_OK ? edt::layout_for(r->H, r->W, true, stack).total : 0;
    if (c == EDT_OK && edt::Arena::round(bytes) > s->alloc.size()) c = EDT_ERR_TOO_LARGE;
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (c == EDT_ERR_TOO_LARGE) s->st.rejected_too_large += 1;
        if (c != EDT_OK) return c;
        if (s->stop) return EDT_ERR_INVALID_ARG;
        if (s->live >= (size_t)s->cfg.max_inflight) {
            s->st.rejected_busy += 1;
            return EDT_ERR_BUSY;
        }
        ev = take_event(s);
        if (!ev) return EDT_ERR_DEVICE;
        s->live += 1;  // reserved until queued below (or given back)
    }
    Req q;
    q.r = *r;
    q.bytes = bytes;
    q.off = 0;
    q.ready = ev;
    const bool rec = hipEventRecord(ev, reinterpret_cast<hipStream_t>(r->stream)) == hipSuccess;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!rec) {
            s->events.push_back(ev);
            s->live -= 1;
            return EDT_ERR_DEVICE;
        }
        q.t0 = Clock::now();
        if (!s->any) {
            s->any = true;
            s->t_first = q.t0;
        }
        q.ticket = s->book.issue();
        s->queue.push_back(q);
        s->st.submitted += 1;
        *ticket = q.ticket;
    }
    s->wake.notify_one();
    return EDT_OK;
}

edt_status edt_serve_poll(edt_server* s, uint64_t ticket, int32_t* done) {
    if (!s || !done) return EDT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->book.known(ticket)) return EDT_ERR_INVALID_ARG;
    const int32_t v = s->book.status(ticket);
    *done = v != kPending;
    return v == kPending ? EDT_OK : v;
}

edt_status edt_serve_wait(edt_server* s, uint64_t ticket, int64_t timeout_ns) {
    if (!s) return EDT_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->book.known(ticket)) return EDT_ERR_INVALID_ARG;
    auto ready = [&] { return s->book.status(ticket) != kPending; };
    if (timeout_ns < 0) {
        s->done_cv.wait(lk, ready);
    } else if (!s->done_cv.wait_for(lk, std::chrono::nanoseconds(timeout_ns), ready)) {
        return EDT_ERR_NOT_READY;
    }
    return s->book.status(ticket);
}

edt_status edt_serve_stats(edt_server* s, edt_serve_counters* out) {
    if (!s || !out) return EDT_ERR_INVALID_ARG;
    // copy the (bounded) latency window under the lock, sort outside it: the
    // scheduler retires requests and admits new ones under the same lock
    std::vector<double> lat;
    edt_serve_counters c;
    double span = 0.0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        c = s->st;
        lat = s->book.window();
        const uint64_t n = s->book.completed();
        c.mean_ns = n ? s->book.latency_sum() / (double)n : 0.0;
        c.max_ns = s->book.latency_max();
        if (s->any && s->st.done > 0)
            span = std::chrono::duration<double>(s->t_last - s->t_first).count();
    }
    c.p50_ns = edt::percentile(lat, 0.50);
    c.p99_ns = edt::percentile(lat, 0.99);
    c.gpix_per_s = span > 0.0 ? (double)c.pixels_done / span / 1e9 : 0.0;
    *out = c;
    return EDT_OK;
}

edt_status edt_serve_destroy(edt_server* s) {
    if (!s) return EDT_ERR_INVALID_ARG;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->wake.notify_all();
    if (s->th.joinable()) s->th.join();
    const edt_status st = s->st.failed > 0 ? EDT_ERR_DEVICE : EDT_OK;
    destroy_parts(s);
    delete s;
    return st;
}

}  // extern "C"
