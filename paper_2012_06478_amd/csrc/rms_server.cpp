// Serving runtime: continuous batching of simulation requests on one GPU.
//
// Scheduling is per slice of steps (iteration-level batching).  One host
// thread owns the device work:
//   1. admit pending requests in arrival order while their device memory fits
//      the budget (buffers allocated and inputs uploaded on the server's
//      stream);
//   2. build one work list per group of admitted requests that share
//      precision, label width, shape count and whether membranes absorb: a
//      block per 256 walkers of each
//      request, each advancing its walkers from the request's current step by
//      the slice length (or to the end);
//   3. run the packed walk launches (walker states stay in HBM between
//      slices), time them with HIP events;
//   4. reduce every request that reached its last step (fixed-order fp64
//      kernels on its own buffers), copy its results to the host, free its
//      memory and wake its waiters.
// Requests submitted during a slice are admitted before the next one, so
// their walkers share launches with requests already running.
#include <hip/hip_runtime.h>

#include <algorithm>
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

struct Request {
    rms_ticket id = 0;
    rms::RunSetup setup;  // holds copies of every input array
    rms::DeviceRun dev;
    size_t bytes = 0;
    int64_t steps_done = 0;
    enum State { kPending, kActive, kDone, kFailed } state = kPending;
    int rc = RMS_OK;
    std::string err;
    std::vector<double> res;
    clock_type::time_point t_submit, t_admit, t_done;
};

}  // namespace

struct rms_server {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    size_t budget = 0, in_use = 0;
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
    // device work-list buffers, grown as needed (worker thread only)
    rms::PackedItem* d_items = nullptr;
    size_t items_cap = 0;
    rms::WalkPlan* d_plans = nullptr;
    size_t plans_cap = 0;

    void loop();
    void finish(Request* r, int rc, const std::string& err);
};

namespace {

template <typename T>
hipError_t grow(T** p, size_t* cap, size_t need, hipStream_t s) {
    if (need <= *cap) return hipSuccess;
    if (*p) {
        hipStreamSynchronize(s);
        hipFree(*p);
        *p = nullptr;
    }
    size_t n = std::max<size_t>(need, 2 * *cap);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T));
    *cap = e == hipSuccess ? n : 0;
    return e;
}

}  // namespace

// Called by the worker with the lock NOT held.
void rms_server::finish(Request* r, int rc, const std::string& err) {
    r->dev.release();
    std::lock_guard<std::mutex> lk(m);
    in_use -= r->bytes;
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

void rms_server::loop() {
    hipSetDevice(device);
    std::vector<Request*> admit;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(m);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !active.empty(); });
            if (stop) break;
            while (!pending.empty() && in_use + pending.front()->bytes <= budget) {
                Request* r = pending.front();
                pending.pop_front();
                in_use += r->bytes;
                admit.push_back(r);
            }
        }
        for (Request* r : admit) {
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
        if (active.empty()) continue;  // active is only touched by this thread

        // slice length
        int64_t walkers = 0;
        for (Request* r : active) walkers += r->setup.n_walkers;
        int64_t S = slice_steps;
        if (S <= 0) S = std::max<int64_t>(64, std::min<int64_t>(1 << 20, 4000000000LL / walkers));
        S = (S + 3) / 4 * 4;  // slices start on a multiple of 4 steps (both Philox streams)

        // one packed launch per (precision, label width, shape count, absorbing)
        std::map<std::tuple<int, int, int, bool>, std::vector<Request*>> groups;
        for (Request* r : active)
            groups[{r->setup.precision, r->setup.sub->dev_label_bytes, r->setup.n_shapes,
                    !r->setup.thr_mt.empty()}]
                .push_back(r);
        std::vector<rms::WalkPlan> plans;
        std::vector<rms::PackedItem> items;
        // key, item range
        std::vector<std::tuple<int, int, int, bool, size_t, size_t>> launches_todo;
        std::vector<int64_t> step_end(active.size());
        std::map<Request*, size_t> index;
        for (size_t i = 0; i < active.size(); ++i) index[active[i]] = i;
        for (auto& g : groups) {
            const size_t first = items.size();
            for (Request* r : g.second) {
                const int plan = static_cast<int>(plans.size());
                plans.push_back(r->dev.wp);
                const int64_t b = r->steps_done;
                const int64_t e = std::min(r->setup.n_steps, b + S);
                step_end[index[r]] = e;
                // slot block k of an ordered run belongs on XCD k mod 8: start the
                // run at a launch block index that is a multiple of 8 (the filler
                // items' slots lie past the run's slots, so their threads exit)
                const int64_t n_slots = r->dev.wp.n_slots;
                if (r->dev.wp.order)
                    while ((items.size() - first) % 8 != 0)
                        items.push_back(rms::PackedItem{n_slots, plan, static_cast<uint32_t>(b),
                                                        static_cast<uint32_t>(e), 0u});
                for (int64_t w = 0; w < n_slots; w += rms::kBlock)
                    items.push_back(rms::PackedItem{w, plan, static_cast<uint32_t>(b),
                                                    static_cast<uint32_t>(e), 0u});
            }
            launches_todo.emplace_back(std::get<0>(g.first), std::get<1>(g.first),
                                       std::get<2>(g.first), std::get<3>(g.first), first,
                                       items.size() - first);
        }
        hipError_t e = grow(&d_items, &items_cap, items.size(), stream);
        if (e == hipSuccess) e = grow(&d_plans, &plans_cap, plans.size(), stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_items, items.data(), items.size() * sizeof(rms::PackedItem),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_plans, plans.data(), plans.size() * sizeof(rms::WalkPlan),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipEventRecord(ev0, stream);
        for (auto& L : launches_todo) {
            if (e != hipSuccess) break;
            e = rms::launch_walk_packed(d_items + std::get<4>(L), static_cast<int>(std::get<5>(L)),
                                        d_plans, std::get<0>(L), std::get<1>(L), std::get<2>(L),
                                        std::get<3>(L), stream);
        }
        if (e == hipSuccess) e = hipEventRecord(ev1, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        float ms = 0.0f;
        if (e == hipSuccess) hipEventElapsedTime(&ms, ev0, ev1);
        {
            std::lock_guard<std::mutex> lk(m);
            ++launches;
            busy_s += ms * 1e-3;
        }
        std::vector<Request*> still;
        for (size_t i = 0; i < active.size(); ++i) {
            Request* r = active[i];
            if (e != hipSuccess) {
                finish(r, RMS_E_DEVICE, std::string("packed walk: ") + hipGetErrorString(e));
                continue;
            }
            r->steps_done = step_end[i];
            if (r->steps_done < r->setup.n_steps) {
                still.push_back(r);
                continue;
            }
            r->res.assign(r->setup.n_res, 0.0);
            hipError_t er = rms::launch_reduce(r->dev.rp, stream);
            if (er == hipSuccess)
                er = hipMemcpyAsync(r->res.data(), r->dev.rp.result, r->res.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, stream);
            if (er == hipSuccess) er = hipStreamSynchronize(stream);
            finish(r, er == hipSuccess ? RMS_OK : RMS_E_DEVICE,
                   er == hipSuccess ? "" : std::string("reduction: ") + hipGetErrorString(er));
        }
        active.swap(still);
    }
    // stopping: fail whatever is left
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
    if (e == hipSuccess) e = hipEventCreate(&s->ev0);
    if (e == hipSuccess) e = hipEventCreate(&s->ev1);
    size_t free_b = 0, total_b = 0;
    if (e == hipSuccess) e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) {
        const int rc = rms::hip_fail("server setup", e);
        if (s->ev1) hipEventDestroy(s->ev1);
        if (s->ev0) hipEventDestroy(s->ev0);
        if (s->stream) hipStreamDestroy(s->stream);
        delete s;
        return rc;
    }
    s->budget = mem_budget_bytes ? mem_budget_bytes : free_b / 4 * 3;
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
    hipSetDevice(srv->device);
    hipStreamSynchronize(srv->stream);
    if (srv->d_items) hipFree(srv->d_items);
    if (srv->d_plans) hipFree(srv->d_plans);
    hipEventDestroy(srv->ev0);
    hipEventDestroy(srv->ev1);
    hipStreamDestroy(srv->stream);
    delete srv;
}

}  // extern "C"
