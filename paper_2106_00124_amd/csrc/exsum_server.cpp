// exsum_server.cpp -- serving form: continuous admission of excluded-sum
// requests by HBM budget and stream slots, with their work overlapping on
// the device.
//
// Paper: Xu, Fraser, Leiserson, "Multidimensional Included and Excluded Sums"
// (SIAM ACDA 2021, arXiv 2106.00124).
//
// A server owns one device arena of `hbm_budget` bytes, carved by a first-fit
// free list (256-byte granules, coalescing frees), and `max_inflight` HIP
// streams.  Requests queue in arrival order; a dispatcher thread admits the
// head of the queue as soon as its bytes (outputs + workspace [+ input when
// the server generates it]) fit the free arena and a stream is idle, enqueues
// its work on that stream (exs_run, the plain path) and records an event.
// Later arrivals are admitted while earlier ones still run, so requests
// overlap on the device.  The dispatcher polls the events; a request's
// latency runs from submit to the detection of its completion.  Memory is
// returned when the client releases the request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "exsum_internal.hpp"

namespace exs {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, cap) with coalescing.
struct FreeList {
    std::map<size_t, size_t> free;  // offset -> size
    size_t cap = 0, used = 0;
    void init(size_t c) {
        cap = c;
        free.clear();
        free[0] = c;
        used = 0;
    }
    static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round(std::max<size_t>(bytes, 1));
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free.erase(it);
                if (rest) free[noff] = rest;
                used += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(std::max<size_t>(bytes, 1));
        used -= bytes;
        auto it = free.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t ticket;
    exs_job job;
    bool generate = false;  // the server fills the input itself
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit: the input is written
    int fill_kind = 0;
    uint64_t seed = 0;
    int64_t lo = 0, hi = 0;
    size_t in_bytes = 0, out_bytes = 0, ws_bytes = 0, total = 0;
    size_t off = 0;
    int slot = -1;
    bool launched = false;  // its work and completion event are enqueued
    enum { QUEUED, RUNNING, DONE, FAILED } state = QUEUED;
    Clock::time_point t_submit, t_done;
    double latency_ms = 0;
    int64_t elems = 0;
};

}  // namespace exs

using namespace exs;

struct exs_server {
    size_t budget = 0;
    char* arena = nullptr;
    FreeList fl;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<uint64_t> slot_owner;  // 0 = idle
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    std::atomic<bool> stop{false};
    std::thread worker;
    int device = 0;
    // events recycled for submit/release ordering, and arena ranges whose
    // release waits for work the caller enqueued on its own stream
    std::vector<hipEvent_t> spare_events;
    struct Deferred {
        size_t off, bytes;
        hipEvent_t ev;
    };
    std::vector<Deferred> deferred;
    // statistics
    std::vector<double> lat;
    int64_t completed = 0, failed = 0, max_queue = 0, elems_done = 0;
    size_t peak_bytes = 0;
    bool have_first = false;
    Clock::time_point t_first, t_last;
    std::string last_error;
};

namespace exs {

static size_t req_bytes(Request& r) {
    const size_t es = dtype_size(r.job.dtype);
    int64_t n = 1;
    for (int i = 0; i < r.job.d; ++i) n *= r.job.dims[i];
    r.elems = n;
    size_t outs = 0;
    if (r.job.mode & EXS_INCLUDED) outs += FreeList::round((size_t)n * es);
    if (r.job.mode & EXS_EXCLUDED) outs += FreeList::round((size_t)n * es);
    r.out_bytes = outs;
    r.in_bytes = r.generate ? FreeList::round((size_t)n * es) : 0;
    size_t ws = 0;
    exs_job probe = r.job;
    if (exs_workspace_size(&probe, &ws) != EXS_OK) ws = 0;
    r.ws_bytes = FreeList::round(ws);
    r.total = r.in_bytes + r.out_bytes + r.ws_bytes;
    return r.total;
}

// An event from the pool (lock held), or a new one.
static hipEvent_t take_event(exs_server* s) {
    if (!s->spare_events.empty()) {
        hipEvent_t e = s->spare_events.back();
        s->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// Return the arena ranges whose caller-stream event has completed (lock held).
static bool reap_deferred(exs_server* s) {
    bool any = false;
    for (size_t i = 0; i < s->deferred.size();) {
        auto& d = s->deferred[i];
        if (hipEventQuery(d.ev) == hipSuccess) {
            s->fl.release(d.off, d.bytes);
            s->spare_events.push_back(d.ev);
            d = s->deferred.back();
            s->deferred.pop_back();
            any = true;
        } else {
            ++i;
        }
    }
    return any;
}

// Admit queued requests (FIFO) while memory and a stream allow: assign
// arena space and a stream slot.  Called with the lock held; the returned
// requests are launched after the lock is dropped.
static std::vector<Request*> admit(exs_server* s) {
    std::vector<Request*> go;
    while (!s->queue.empty()) {
        Request& r = s->reqs[s->queue.front()];
        int slot = -1;
        for (size_t i = 0; i < s->slot_owner.size(); ++i)
            if (s->slot_owner[i] == 0) { slot = (int)i; break; }
        if (slot < 0) break;
        size_t off = 0;
        if (!s->fl.alloc(r.total, &off)) break;  // the head of the line waits for memory
        s->queue.pop_front();
        r.off = off;
        r.slot = slot;
        r.launched = false;
        r.state = Request::RUNNING;
        s->slot_owner[slot] = r.ticket;
        s->peak_bytes = std::max(s->peak_bytes, s->fl.used);
        char* base = s->arena + off;
        const size_t es = dtype_size(r.job.dtype);
        char* outp = base + r.in_bytes;
        if (r.generate) r.job.in_dev = base;
        r.job.inc_out_dev = nullptr;
        r.job.exc_out_dev = nullptr;
        if (r.job.mode & EXS_INCLUDED) {
            r.job.inc_out_dev = outp;
            outp += FreeList::round((size_t)r.elems * es);
        }
        if (r.job.mode & EXS_EXCLUDED) r.job.exc_out_dev = outp;
        go.push_back(&r);
    }
    return go;
}

// Enqueue a request's work on its stream (no lock held).
static exs_status launch(exs_server* s, Request& r) {
    char* ws = s->arena + r.off + r.in_bytes + r.out_bytes;
    hipStream_t st = s->streams[r.slot];
    exs_status rc = EXS_OK;
    if (r.ready && hipStreamWaitEvent(st, r.ready, 0) != hipSuccess)
        rc = set_error(EXS_EDEVICE, "hipStreamWaitEvent failed");
    if (rc == EXS_OK && r.generate)
        rc = exs_fill((void*)r.job.in_dev, r.elems, r.job.dtype, r.fill_kind, r.seed, r.lo, r.hi, st);
    if (rc == EXS_OK) rc = exs_run(&r.job, ws, r.ws_bytes, st);
    if (rc == EXS_OK && hipEventRecord(s->events[r.slot], st) != hipSuccess)
        rc = set_error(EXS_EDEVICE, "hipEventRecord failed");
    return rc;
}

// Retire finished requests; called with the lock held.
static bool retire(exs_server* s) {
    bool any = false;
    for (size_t i = 0; i < s->slot_owner.size(); ++i) {
        const uint64_t t = s->slot_owner[i];
        if (!t) continue;
        Request& r = s->reqs[t];
        if (!r.launched) continue;
        if (hipEventQuery(s->events[i]) != hipSuccess) continue;
        r.t_done = Clock::now();
        r.state = Request::DONE;
        r.latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
        s->slot_owner[i] = 0;
        s->lat.push_back(r.latency_ms);
        ++s->completed;
        s->elems_done += r.elems;
        s->t_last = r.t_done;
        any = true;
    }
    return any;
}

static void worker_loop(exs_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->stop.load()) {
        const bool busy = std::any_of(s->slot_owner.begin(), s->slot_owner.end(),
                                      [](uint64_t t) { return t != 0; });
        if (!busy && s->queue.empty() && s->deferred.empty()) {
            s->cv.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        const bool reaped = reap_deferred(s);
        const bool freed = retire(s) || reaped;
        std::vector<Request*> go = admit(s);
        if (freed) s->cv.notify_all();
        lk.unlock();
        std::vector<std::pair<Request*, exs_status>> res;
        for (Request* r : go) res.emplace_back(r, launch(s, *r));
        // while work is in flight the worker polls the slot events: a timed
        // sleep would add the kernel timer's slack to every request's latency
        if (go.empty()) std::this_thread::yield();
        lk.lock();
        for (auto& pr : res) {
            Request& r = *pr.first;
            if (r.ready) {
                // the wait is enqueued (or the launch failed): the event can be reused
                s->spare_events.push_back(r.ready);
                r.ready = nullptr;
            }
            if (pr.second == EXS_OK) {
                r.launched = true;
            } else {
                // the slot's stream may hold part of the work: wait for it
                (void)hipStreamSynchronize(s->streams[r.slot]);
                s->last_error = exs_last_error();
                r.state = Request::FAILED;
                s->slot_owner[r.slot] = 0;
                s->fl.release(r.off, r.total);
                ++s->failed;
            }
        }
    }
}

// Whether the queue head fits a free range of the arena (lock held).
static bool head_fits(exs_server* s) {
    if (s->queue.empty()) return true;
    const size_t need = FreeList::round(std::max<size_t>(s->reqs[s->queue.front()].total, 1));
    for (const auto& f : s->fl.free)
        if (f.second >= need) return true;
    return false;
}

static exs_status submit_common(exs_server* s, Request&& r, uint64_t* ticket, bool wait_caller,
                                void* caller_stream) {
    exs_status st = validate_job(&r.job, false);
    if (st != EXS_OK) return st;
    if (!r.generate && !r.job.in_dev) return set_error(EXS_EINVAL, "in_dev is NULL");
    if (req_bytes(r) > s->budget)
        return set_error(EXS_ENOMEM, "request larger than the whole HBM budget");
    std::lock_guard<std::mutex> g(s->mu);
    if (wait_caller) {
        // the request's work starts only after the caller's stream has reached
        // this point (the input is written there)
        r.ready = take_event(s);
        if (!r.ready || hipEventRecord(r.ready, (hipStream_t)caller_stream) != hipSuccess) {
            if (r.ready) s->spare_events.push_back(r.ready);
            return set_error(EXS_EDEVICE, "cannot record the input event on the caller's stream");
        }
    }
    r.ticket = s->next_ticket++;
    r.t_submit = Clock::now();
    if (!s->have_first) {
        s->have_first = true;
        s->t_first = r.t_submit;
    }
    const uint64_t t = r.ticket;
    s->reqs.emplace(t, std::move(r));
    s->queue.push_back(t);
    s->max_queue = std::max<int64_t>(s->max_queue, (int64_t)s->queue.size());
    *ticket = t;
    s->cv.notify_all();
    return EXS_OK;
}

}  // namespace exs

extern "C" {

exs_status exs_server_create(size_t hbm_budget, int32_t max_inflight, exs_server** out) {
    if (!out) return set_error(EXS_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget < 4096 || max_inflight < 1 || max_inflight > 64)
        return set_error(EXS_EINVAL, "need hbm_budget >= 4096 and 1 <= max_inflight <= 64");
    exs_server* s = new (std::nothrow) exs_server();
    if (!s) return set_error(EXS_ENOMEM, "out of host memory");
    (void)hipGetDevice(&s->device);
    s->budget = FreeList::round(hbm_budget);
    if (hipMalloc((void**)&s->arena, s->budget) != hipSuccess) {
        delete s;
        return set_error(EXS_ENOMEM, "cannot allocate the serving arena");
    }
    s->fl.init(s->budget);
    for (int i = 0; i < max_inflight; ++i) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            exs_server_destroy(s);
            return set_error(EXS_EDEVICE, "cannot create streams/events");
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
        s->slot_owner.push_back(0);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return EXS_OK;
}

exs_status exs_server_submit(exs_server* s, const exs_job* job, void* stream, uint64_t* ticket) {
    if (!s || !job || !ticket) return set_error(EXS_EINVAL, "NULL argument");
    Request r;
    r.job = *job;
    return submit_common(s, std::move(r), ticket, true, stream);
}

exs_status exs_server_submit_generated(exs_server* s, const exs_job* job, int32_t fill_kind,
                                       uint64_t seed, int64_t lo, int64_t hi, uint64_t* ticket) {
    if (!s || !job || !ticket) return set_error(EXS_EINVAL, "NULL argument");
    const bool int_fill = fill_kind == 1;
    const bool ok = int_fill ? (job->dtype == EXS_I32 || job->dtype == EXS_I64)
                             : job->dtype == EXS_F32;
    if (!ok) return set_error(EXS_EINVAL, "fill kind does not match the job's dtype");
    Request r;
    r.job = *job;
    r.generate = true;
    r.fill_kind = fill_kind;
    r.seed = seed;
    r.lo = lo;
    r.hi = hi;
    return submit_common(s, std::move(r), ticket, false, nullptr);
}

exs_status exs_server_poll(exs_server* s, uint64_t ticket, const void** inc_dev,
                           const void** exc_dev, double* latency_ms) {
    if (!s) return set_error(EXS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(EXS_ENOTFOUND, "unknown ticket");
    Request& r = it->second;
    if (r.state == Request::FAILED)
        return set_error(EXS_EDEVICE, "request failed: " + s->last_error);
    if (r.state != Request::DONE) return EXS_ENOTREADY;
    if (inc_dev) *inc_dev = r.job.inc_out_dev;
    if (exc_dev) *exc_dev = r.job.exc_out_dev;
    if (latency_ms) *latency_ms = r.latency_ms;
    return EXS_OK;
}

exs_status exs_server_input(exs_server* s, uint64_t ticket, const void** in_dev) {
    if (!s || !in_dev) return set_error(EXS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(EXS_ENOTFOUND, "unknown ticket");
    if (it->second.state != Request::DONE) return EXS_ENOTREADY;
    *in_dev = it->second.job.in_dev;
    return EXS_OK;
}

exs_status exs_server_drain(exs_server* s) {
    if (!s) return set_error(EXS_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        const bool busy = std::any_of(s->slot_owner.begin(), s->slot_owner.end(),
                                      [](uint64_t t) { return t != 0; }) ||
                          !s->deferred.empty();
        if (!busy && s->queue.empty()) return EXS_OK;
        if (!busy && !head_fits(s))
            return set_error(EXS_EAGAIN,
                             "queue blocked: release completed requests to free the arena");
        s->cv.wait_for(lk, std::chrono::milliseconds(1));
    }
}

exs_status exs_server_release(exs_server* s, uint64_t ticket, void* stream) {
    if (!s) return set_error(EXS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(EXS_ENOTFOUND, "unknown ticket");
    Request& r = it->second;
    if (r.state == Request::QUEUED || r.state == Request::RUNNING)
        return set_error(EXS_ENOTREADY, "request still pending");
    if (r.state == Request::DONE) {
        // the caller may still read the outputs on its stream: the range goes
        // back to the arena once that stream passes this point
        hipEvent_t ev = take_event(s);
        if (!ev || hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
            if (ev) s->spare_events.push_back(ev);
            return set_error(EXS_EDEVICE, "cannot record the release event on the caller's stream");
        }
        s->deferred.push_back({r.off, r.total, ev});
    }
    s->reqs.erase(it);
    s->cv.notify_all();
    return EXS_OK;
}

exs_status exs_server_stats(exs_server* s, double* p50_ms, double* p99_ms, double* req_per_s,
                            double* gelem_per_s, int64_t* completed, int64_t* max_queue,
                            int64_t* peak_bytes) {
    if (!s) return set_error(EXS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        size_t i = (size_t)std::ceil(p * (double)v.size()) ;
        if (i > 0) --i;
        if (i >= v.size()) i = v.size() - 1;
        return v[i];
    };
    double span = 0;
    if (s->have_first && s->completed)
        span = std::chrono::duration<double>(s->t_last - s->t_first).count();
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (req_per_s) *req_per_s = span > 0 ? (double)s->completed / span : 0.0;
    if (gelem_per_s) *gelem_per_s = span > 0 ? (double)s->elems_done / span / 1e9 : 0.0;
    if (completed) *completed = s->completed;
    if (max_queue) *max_queue = s->max_queue;
    if (peak_bytes) *peak_bytes = (int64_t)s->peak_bytes;
    return EXS_OK;
}

void exs_server_destroy(exs_server* s) {
    if (!s) return;
    s->stop.store(true);
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (auto ev : s->events) (void)hipEventDestroy(ev);
    for (auto& d : s->deferred) {
        (void)hipEventSynchronize(d.ev);
        (void)hipEventDestroy(d.ev);
    }
    for (auto ev : s->spare_events) (void)hipEventDestroy(ev);
    for (auto& kv : s->reqs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    if (s->arena) (void)hipFree(s->arena);
    delete s;
}

}  // extern "C"
