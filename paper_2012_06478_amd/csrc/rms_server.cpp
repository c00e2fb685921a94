// Serving runtime: continuous batching of simulation requests on one GPU.
//
// Scheduling is per slice of steps (iteration-level batching).  One host
// thread owns the device work and keeps the device fed: it enqueues slice
// k + 1 before it waits for slice k, so the stream always holds the next
// launch while the host handles the previous one.  Per iteration it
//   1. admits pending requests in arrival order while their device memory
//      fits the budget (buffers allocated from the library's stream-ordered
//      pool and inputs uploaded on the server's stream, walker order built);
//   2. if fewer than kDepth slices are in flight, enqueues the next slice:
//      one packed launch per group of admitted requests that share
//      precision, label width, shape count and whether membranes absorb,
//      with a block per 256 walkers of each request advancing them from the
//      request's scheduled step by the slice length (or to the end; requests
//      that end early come last in their launch), then, for every request
//      whose last steps the slice holds, its fixed-order fp64 reduction, the
//      copy of its results to a pinned host block and the stream-ordered
//      release of its device memory;
//   3. otherwise waits for the oldest slice in flight and completes the
//      requests it finished (their results are already in host memory).
// Requests submitted while slices run are admitted before the next slice is
// built, so their walkers share launches with requests already running, and
// the memory that finished requests free is admitted again in stream order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "rms_host.h"

namespace {

using clock_type = std::chrono::steady_clock;

double seconds_since(clock_type::time_point t0, clock_type::time_point t) {
    return std::chrono::duration<double>(t - t0).count();
}

// Slices in flight at once: the one running and the one queued behind it.
constexpr int kDepth = 2;

// RMS_OPT_SERVER_WALKERS (0: automatic), read when a server is created.
std::atomic<int64_t> g_server_walkers{0};

// Automatic walker slots: sixteen rounds of the resident waves of the mixed
// walker (six per SIMD).  With every queued request admitted, the slices
// shrink to their 64-step minimum and their walkers read the labels of many
// substrates; with a cap, a slice is long enough that moving the walker
// states between slices costs little, while every launch still fills the
// device.
int64_t auto_walker_slots(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        cus <= 0)
        cus = 256;
    return int64_t(cus) * 4 * 6 * 64 * 16;
}
// Largest result record of a request: kAccFixed + 2 n_sig + 2 n_dirs doubles.
constexpr size_t kResMax = rms::kAccFixed + 2 * RMS_MAX_SIGNALS + 2 * RMS_MAX_SIGNALS;

struct Request {
    rms_ticket id = 0;
    rms::RunSetup setup;  // holds copies of every input array
    rms::DeviceRun dev;
    size_t bytes = 0;
    int64_t steps_sched = 0;   // steps enqueued on the device
    bool last_sched = false;   // the slice with its last steps is enqueued
    bool admitted = false;     // holds walker slots and memory of the budget
    double* h_res = nullptr;   // pinned block its results are copied to
    enum State { kPending, kActive, kDone, kFailed } state = kPending;
    int rc = RMS_OK;
    std::string err;
    std::vector<double> res;
    clock_type::time_point t_submit, t_admit, t_done;
};

// Device work list of one slice: items and plans, grown as needed
// (stream-ordered, so a buffer is replaced only behind the work that read it).
struct WorkBuffer {
    rms::PackedItem* items = nullptr;
    size_t items_cap = 0;
    rms::WalkPlan* plans = nullptr;
    size_t plans_cap = 0;
};

struct Slice {
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    std::vector<Request*> members;    // every request with steps in the slice
    std::vector<Request*> finishing;  // those whose last steps it holds
    std::vector<rms::PackedItem> items;  // host copies, alive until the slice is done
    std::vector<rms::WalkPlan> plans;
    hipError_t err = hipSuccess;
    std::string what;
};

}  // namespace

struct rms_server {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t events[2 * kDepth] = {};
    size_t budget = 0, in_use = 0;
    int64_t walker_slots = 0, walkers_in_use = 0;  // of the admitted requests
    int slice_steps = 0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> active;
    std::map<rms_ticket, std::unique_ptr<Request>> all;
    rms_ticket next_id = 1;
    bool stop = false;
    std::thread worker;
    // statistics
    int64_t submitted = 0, completed = 0, failed = 0, launches = 0, walker_steps = 0;
    double busy_s = 0.0;
    // worker thread only
    WorkBuffer bufs[kDepth];
    int next_buf = 0;
    std::vector<double*> pinned_free, pinned_all;

    void loop();
    void enqueue_slice(std::deque<Slice>& inflight);
    void complete_oldest(std::deque<Slice>& inflight);
    void finish(Request* r, int rc, const std::string& err);
    void free_device(Request* r);
};

namespace {

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t need, hipStream_t s) {
    if (need <= *cap) return hipSuccess;
    if (*p) {
        (void)hipFreeAsync(*p, s);
        *p = nullptr;
    }
    const size_t n = std::max<size_t>(need, 2 * *cap);
    void* q = nullptr;
    hipError_t e = rms::run_malloc(&q, n * sizeof(T), s);
    *p = static_cast<T*>(q);
    *cap = e == hipSuccess ? n : 0;
    return e;
}

}  // namespace

// Stream-ordered release of a request's device memory (behind every launch
// already enqueued that reads it).
void rms_server::free_device(Request* r) {
    for (void* p : r->dev.ptrs) (void)hipFreeAsync(p, stream);
    r->dev.ptrs.clear();
}

// Worker thread; the lock is NOT held.
void rms_server::finish(Request* r, int rc, const std::string& err) {
    free_device(r);
    if (r->h_res) {
        if (rc == RMS_OK) r->res.assign(r->h_res, r->h_res + r->setup.n_res);
        if (static_cast<size_t>(r->setup.n_res) <= kResMax) pinned_free.push_back(r->h_res);
        r->h_res = nullptr;
    }
    std::lock_guard<std::mutex> lk(m);
    if (r->admitted) {  // requests still pending at destruction hold nothing
        in_use -= r->bytes;
        walkers_in_use -= r->setup.n_walkers;
        r->admitted = false;
    }
    r->rc = rc;
    r->err = err;
    r->t_done = clock_type::now();
    r->state = rc == RMS_OK ? Request::kDone : Request::kFailed;
    if (rc == RMS_OK) {
        ++completed;
        walker_steps += r->setup.n_walkers * r->setup.n_steps;
    } else {
        ++failed;
    }
    cv_done.notify_all();
}

void rms_server::enqueue_slice(std::deque<Slice>& inflight) {
    inflight.emplace_back();
    Slice& sl = inflight.back();
    sl.ev_begin = events[2 * next_buf];
    sl.ev_end = events[2 * next_buf + 1];
    WorkBuffer& wb = bufs[next_buf];
    next_buf = (next_buf + 1) % kDepth;

    // slice length
    int64_t walkers = 0;
    for (Request* r : active)
        if (!r->last_sched) walkers += r->setup.n_walkers;
    int64_t S = slice_steps;
    if (S <= 0) S = std::max<int64_t>(64, std::min<int64_t>(1 << 20, 4000000000LL / walkers));
    S = (S + 3) / 4 * 4;  // slices start on a multiple of 4 steps (both Philox streams)

    // one packed launch per (precision, label width, shape count, absorbing)
    std::map<std::tuple<int, int, int, bool>, std::vector<Request*>> groups;
    for (Request* r : active)
        if (!r->last_sched)
            groups[{r->setup.precision, r->setup.sub->dev_label_bytes, r->setup.n_shapes,
                    !r->setup.thr_mt.empty()}]
                .push_back(r);
    std::vector<std::tuple<int, int, int, bool, size_t, size_t>> todo;  // key, item range
    for (auto& g : groups) {
        // requests that run the whole slice first, those that end early last
        std::stable_sort(g.second.begin(), g.second.end(), [S](Request* a, Request* b) {
            return std::min(S, a->setup.n_steps - a->steps_sched) >
                   std::min(S, b->setup.n_steps - b->steps_sched);
        });
        const size_t first = sl.items.size();
        for (Request* r : g.second) {
            const int plan = static_cast<int>(sl.plans.size());
            sl.plans.push_back(r->dev.wp);
            const int64_t b = r->steps_sched;
            const int64_t e = std::min(r->setup.n_steps, b + S);
            // slot block k of an ordered run belongs on XCD k mod 8: start the
            // run at a launch block index that is a multiple of 8 (the filler
            // items' slots lie past the run's slots, so their threads exit)
            const int64_t n_slots = r->dev.wp.n_slots;
            if (r->dev.wp.order)
                while ((sl.items.size() - first) % 8 != 0)
                    sl.items.push_back(rms::PackedItem{n_slots, plan, static_cast<uint32_t>(b),
                                                       static_cast<uint32_t>(e), 0u});
            for (int64_t w = 0; w < n_slots; w += rms::kBlock)
                sl.items.push_back(rms::PackedItem{w, plan, static_cast<uint32_t>(b),
                                                   static_cast<uint32_t>(e), 0u});
            r->steps_sched = e;
            sl.members.push_back(r);
            if (e == r->setup.n_steps) {
                r->last_sched = true;
                sl.finishing.push_back(r);
            }
        }
        todo.emplace_back(std::get<0>(g.first), std::get<1>(g.first), std::get<2>(g.first),
                          std::get<3>(g.first), first, sl.items.size() - first);
    }
    hipError_t e = grow(&wb.items, &wb.items_cap, sl.items.size(), stream);
    if (e == hipSuccess) e = grow(&wb.plans, &wb.plans_cap, sl.plans.size(), stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(wb.items, sl.items.data(), sl.items.size() * sizeof(rms::PackedItem),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(wb.plans, sl.plans.data(), sl.plans.size() * sizeof(rms::WalkPlan),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(sl.ev_begin, stream);
    for (auto& L : todo) {
        if (e != hipSuccess) break;
        e = rms::launch_walk_packed(wb.items + std::get<4>(L), static_cast<int>(std::get<5>(L)),
                                    wb.plans, std::get<0>(L), std::get<1>(L), std::get<2>(L),
                                    std::get<3>(L), stream);
    }
    if (e != hipSuccess) sl.what = "packed walk";
    for (Request* r : sl.finishing) {
        if (e != hipSuccess) break;
        e = rms::launch_reduce(r->dev.rp, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r->h_res, r->dev.rp.result, r->setup.n_res * sizeof(double),
                               hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) free_device(r);
        else sl.what = "reduction";
    }
    if (e == hipSuccess) e = hipEventRecord(sl.ev_end, stream);
    sl.err = e;
    {
        std::lock_guard<std::mutex> lk(m);
        launches += static_cast<int64_t>(todo.size());
    }
}

// Completes the oldest slice in flight and drops it.  After a device error
// every admitted request has failed (their device work is in doubt), so the
// slices queued behind no longer refer to live requests: they are waited for
// and dropped as well.
void rms_server::complete_oldest(std::deque<Slice>& inflight) {
    Slice& sl = inflight.front();
    hipError_t e = sl.err;
    if (e == hipSuccess) e = hipEventSynchronize(sl.ev_end);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, sl.ev_begin, sl.ev_end);
    if (e != hipSuccess) {
        const std::string msg = std::string(sl.what.empty() ? "slice" : sl.what) + ": " +
                                hipGetErrorString(e);
        std::vector<Request*> all_active;
        all_active.swap(active);
        for (Request* r : all_active) finish(r, RMS_E_DEVICE, msg);
        inflight.pop_front();
        for (; !inflight.empty(); inflight.pop_front())
            (void)hipEventSynchronize(inflight.front().ev_end);
        return;
    }
    {
        std::lock_guard<std::mutex> lk(m);
        busy_s += ms * 1e-3;
    }
    for (Request* r : sl.finishing) {
        active.erase(std::find(active.begin(), active.end(), r));
        finish(r, RMS_OK, "");
    }
    inflight.pop_front();
}

void rms_server::loop() {
    (void)hipSetDevice(device);
    std::deque<Slice> inflight;
    std::vector<Request*> admit;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(m);
            if (inflight.empty() && active.empty())
                cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            if (stop) break;
            // in arrival order, while the memory budget and the walker slots
            // hold them (a request larger than all the slots runs alone)
            while (!pending.empty() && in_use + pending.front()->bytes <= budget &&
                   (walkers_in_use == 0 ||
                    walkers_in_use + pending.front()->setup.n_walkers <= walker_slots)) {
                Request* r = pending.front();
                pending.pop_front();
                in_use += r->bytes;
                walkers_in_use += r->setup.n_walkers;
                r->admitted = true;
                admit.push_back(r);
            }
        }
        for (Request* r : admit) {
            const bool big = static_cast<size_t>(r->setup.n_res) > kResMax;  // many directions
            if (big || pinned_free.empty()) {
                void* h = nullptr;
                const size_t n = big ? static_cast<size_t>(r->setup.n_res) : kResMax;
                if (hipHostMalloc(&h, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
                    finish(r, RMS_E_OOM, "pinned result buffer");
                    continue;
                }
                pinned_all.push_back(static_cast<double*>(h));
                if (!big) pinned_free.push_back(static_cast<double*>(h));
                else r->h_res = static_cast<double*>(h);
            }
            if (!big) {
                r->h_res = pinned_free.back();
                pinned_free.pop_back();
            }
            int rc = r->dev.create(*r->setup.sub, r->setup, true, stream);
            if (rc == RMS_OK) {
                hipError_t eo = rms::launch_start_try(r->dev.wp, stream);
                if (eo == hipSuccess) eo = rms::launch_order(r->dev.wp, stream);
                if (eo != hipSuccess) rc = rms::hip_fail("walker order", eo);
            }
            if (rc != RMS_OK) {
                finish(r, rc, rms::last_error());
                continue;
            }
            std::lock_guard<std::mutex> lk(m);
            r->state = Request::kActive;
            r->t_admit = clock_type::now();
            active.push_back(r);
        }
        admit.clear();
        const bool work = std::any_of(active.begin(), active.end(),
                                      [](Request* r) { return !r->last_sched; });
        if (work && inflight.size() < static_cast<size_t>(kDepth)) {
            enqueue_slice(inflight);
            continue;
        }
        if (inflight.empty()) continue;
        complete_oldest(inflight);
    }
    // stopping: let the slices in flight end, then fail whatever is left
    while (!inflight.empty()) complete_oldest(inflight);
    std::vector<Request*> left;
    {
        std::lock_guard<std::mutex> lk(m);
        left.assign(pending.begin(), pending.end());
        pending.clear();
    }
    left.insert(left.end(), active.begin(), active.end());
    active.clear();
    for (Request* r : left) finish(r, RMS_E_INVALID_ARG, "server destroyed before completion");
}

namespace rms {
void set_server_walkers(int64_t walkers) {
    g_server_walkers.store(walkers, std::memory_order_relaxed);
}
}  // namespace rms

extern "C" {

int rms_server_create(size_t mem_budget_bytes, int slice_steps, rms_server** out) {
    rms::clear_error();
    if (!out) return rms::fail(RMS_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (slice_steps < 0 || slice_steps == 1)
        return rms::fail(RMS_E_INVALID_ARG, "slice_steps must be 0 or >= 2");
    auto* s = new (std::nothrow) rms_server;
    if (!s) return rms::fail(RMS_E_OOM, "host allocation failed");
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (hipEvent_t& ev : s->events)
        if (e == hipSuccess) e = hipEventCreate(&ev);
    size_t free_b = 0, total_b = 0;
    if (e == hipSuccess) e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) {
        const int rc = rms::hip_fail("server setup", e);
        for (hipEvent_t ev : s->events)
            if (ev) (void)hipEventDestroy(ev);
        if (s->stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return rc;
    }
    s->budget = mem_budget_bytes ? mem_budget_bytes : free_b / 4 * 3;
    const int64_t w = g_server_walkers.load(std::memory_order_relaxed);
    s->walker_slots = w > 0 ? w : auto_walker_slots(s->device);
    s->slice_steps = (slice_steps + 3) / 4 * 4;
    s->worker = std::thread([s] { s->loop(); });
    *out = s;
    return RMS_OK;
}

int rms_server_submit(rms_server* srv, const rms_request* q, rms_ticket* ticket) {
    rms::clear_error();
    if (!srv || !q || !ticket) return rms::fail(RMS_E_INVALID_ARG, "server, request and ticket are required");
    if (q->substrate && q->substrate->device != srv->device)
        return rms::fail(RMS_E_INVALID_ARG, "substrate lives on another device than the server");
    auto r = std::make_unique<Request>();
    const int rc = rms::prepare_run(q->substrate, q->params, q->seed, q->n_walkers, q->n_steps,
                                    q->dt_ms, q->n_shapes, q->waveform, q->n_dirs, q->dirs, q->n_b,
                                    q->bvals, q->precision, r->setup);
    if (rc) return rc;
    r->bytes = rms::device_bytes(r->setup, true);
    r->t_submit = clock_type::now();
    std::lock_guard<std::mutex> lk(srv->m);
    if (r->bytes > srv->budget)
        return rms::fail(RMS_E_BUSY, "request needs " + std::to_string(r->bytes) +
                                         " device bytes, more than the server budget");
    if (srv->stop) return rms::fail(RMS_E_INVALID_ARG, "server is stopping");
    r->id = srv->next_id++;
    *ticket = r->id;
    srv->pending.push_back(r.get());
    srv->all[r->id] = std::move(r);
    ++srv->submitted;
    srv->cv_work.notify_all();
    return RMS_OK;
}

int rms_server_poll(rms_server* srv, rms_ticket ticket, int* done) {
    rms::clear_error();
    if (!srv || !done) return rms::fail(RMS_E_INVALID_ARG, "server and done are required");
    std::lock_guard<std::mutex> lk(srv->m);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return rms::fail(RMS_E_INVALID_ARG, "unknown ticket");
    *done = it->second->state == Request::kDone || it->second->state == Request::kFailed;
    return RMS_OK;
}

int rms_server_wait(rms_server* srv, rms_ticket ticket, double timeout_s, rms_result* out) {
    rms::clear_error();
    if (!srv || !out) return rms::fail(RMS_E_INVALID_ARG, "server and result are required");
    if (out->walker_dump)
        return rms::fail(RMS_E_INVALID_ARG, "walker dumps are not kept for server requests");
    std::unique_lock<std::mutex> lk(srv->m);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return rms::fail(RMS_E_INVALID_ARG, "unknown ticket");
    Request* r = it->second.get();
    auto ready = [&] { return r->state == Request::kDone || r->state == Request::kFailed; };
    if (timeout_s < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
        return rms::fail(RMS_E_TIMEOUT, "request not complete");
    }
    std::unique_ptr<Request> own = std::move(it->second);
    srv->all.erase(it);
    lk.unlock();
    if (own->state == Request::kFailed) return rms::fail(own->rc, own->err);
    rms::fill_result(own->setup, own->res.data(), out);
    out->kernel_ms = 0.0;
    out->walk_kernel = RMS_WALK_PACKED;
    out->wall_s = seconds_since(own->t_submit, own->t_done);
    out->queue_s = seconds_since(own->t_submit, own->t_admit);
    return RMS_OK;
}

int rms_server_stats_get(rms_server* srv, rms_server_stats* out) {
    rms::clear_error();
    if (!srv || !out) return rms::fail(RMS_E_INVALID_ARG, "server and stats are required");
    std::lock_guard<std::mutex> lk(srv->m);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->failed = srv->failed;
    out->pending = static_cast<int64_t>(srv->pending.size());
    int64_t active = 0;
    for (auto& kv : srv->all) active += kv.second->state == Request::kActive;
    out->active = active;
    out->launches = srv->launches;
    out->walker_steps = srv->walker_steps;
    out->busy_s = srv->busy_s;
    out->bytes_in_use = srv->in_use;
    out->bytes_budget = srv->budget;
    return RMS_OK;
}

void rms_server_destroy(rms_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->m);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    (void)hipSetDevice(srv->device);
    for (WorkBuffer& wb : srv->bufs) {
        if (wb.items) (void)hipFreeAsync(wb.items, srv->stream);
        if (wb.plans) (void)hipFreeAsync(wb.plans, srv->stream);
    }
    (void)hipStreamSynchronize(srv->stream);
    for (double* h : srv->pinned_all) (void)hipHostFree(h);
    for (hipEvent_t ev : srv->events) (void)hipEventDestroy(ev);
    (void)hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
