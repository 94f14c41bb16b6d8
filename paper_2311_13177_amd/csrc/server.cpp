// Reconstruction server: continuous batching of requests of mixed sizes on one device.
//
// A worker thread admits queued requests in arrival order while a slot is free and the
// sum of their device bytes stays within the budget; each admitted request keeps its
// optimiser state resident and advances on its own stream, replaying its captured step
// (its own tuned tile shape, the same kernels as alone). The oldest resident requests
// step at a time (as many as fill the device), their work overlapping on it; the worker
// keeps up to kDepth super-steps (kSuperSteps optimiser steps each) enqueued for each,
// with the objective behind the last one, and handles completions in enqueue order,
// topping the queues up as it goes. Requests that arrive while others run are admitted (state
// uploaded) as soon as a slot and memory free up, and start stepping without delay. A
// finished request keeps its device state until vp_server_wait copies the volume and
// renders straight into the caller's buffers on the caller's thread and releases it.
// A request's arithmetic does not depend on the mix it runs in, so its result equals
// the one vp_reconstruct computes for it alone.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "plan.h"
#include "runtime.h"

namespace vp {
namespace {

using Clock = std::chrono::steady_clock;

// Steps per super-step; super-steps kept enqueued per stepping request. Resident
// requests with work still to enqueue step together, the oldest first, up to kStepping
// of them and until their volumes reach kFillVoxels (at least one): a large
// reconstruction saturates the device's memory system on its own, and several at once
// would only thrash each other's caches, while small ones share the device. The others
// wait with their state uploaded.
constexpr int kSuperSteps = 8;
constexpr int kDepth = 2;
constexpr int kStepping = 4;
constexpr uint64_t kFillVoxels = uint64_t(1) << 23;

enum class RState { Queued, Running, Done, Spilling, Collecting };

struct Request {
    uint64_t id = 0;
    const vp_plan* plan = nullptr;
    vp_options opts{};
    std::vector<vp_c64> kspace;
    uint64_t bytes = 0;
    RState state = RState::Queued;
    std::atomic<bool> cancel{false};
    vp_status status = VP_OK;
    double final_loss = 0.0;
    int64_t steps_done = 0;
    Clock::time_point t_submit, t_done;
    std::unique_ptr<vp_session> session;
    // worker bookkeeping while resident
    int64_t queued = 0;        // steps enqueued so far
    int inflight = 0;          // enqueued super-steps not yet waited for
    bool final_sent = false;   // the objective has been enqueued
    bool failed = false;
    vp_status fail_status = VP_OK;
    hipEvent_t ev[kDepth] = {};
    unsigned evi = 0;
    vp_status make_events() {
        for (hipEvent_t& e : ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
                return fail(VP_ERR_DEVICE, "server: hipEventCreate failed");
            }
        return VP_OK;
    }
    void release_events() {
        for (hipEvent_t& e : ev) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
    }
    // results moved to host when the device memory was needed before collection
    std::vector<vp_c64> h_vol, h_proj, h_water, h_fat;
};

struct Inflight {
    Request* r;
    hipEvent_t ev;
    bool final;
    vp_status st;  // status of enqueueing it
};

}  // namespace
}  // namespace vp

using namespace vp;

struct vp_server {
    int device = 0;
    uint64_t budget = 0;
    int max_slots = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, std::unique_ptr<Request>> reqs;
    uint64_t next_id = 1;
    uint64_t used = 0;     // device bytes of admitted requests not yet collected by wait
    bool stop = false;
    std::vector<double> latencies_us;
    Clock::time_point t_first_submit{}, t_last_done{};
    bool any_submit = false;
    std::thread worker;
    void run();
    void mark_done(Request* r, vp_status st, bool count);
};

// Worker thread only; takes the lock.
void vp_server::mark_done(Request* r, vp_status st, bool count) {
    std::lock_guard<std::mutex> lk(mu);
    r->status = st;
    r->state = RState::Done;
    r->t_done = Clock::now();
    if (!r->session) used -= r->bytes;  // nothing left on the device to collect
    if (count) {
        latencies_us.push_back(std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count());
        t_last_done = r->t_done;
    }
    cv_done.notify_all();
}

void vp_server::run() {
    (void)hipSetDevice(device);
    std::vector<Request*> active;  // resident: state on the device, work enqueued or to enqueue
    std::deque<Inflight> fifo;     // enqueued super-steps of every resident request, in order
    for (;;) {
        std::vector<Request*> admit, dropped, spill;
        {
            std::unique_lock<std::mutex> lk(mu);
            // a finished request holds its device memory until collected; if the queue
            // head does not fit, move uncollected results to host to make room
            if (!stop && !queue.empty() && used + reqs[queue.front()]->bytes > budget) {
                for (auto& kv : reqs) {
                    Request* r = kv.second.get();
                    if (r->state == RState::Done && r->session) {
                        r->state = RState::Spilling;
                        spill.push_back(r);
                    }
                }
            }
            // cancelled requests leave once their enqueued work has drained
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel && (*it)->inflight == 0) {
                    dropped.push_back(*it);
                    it = active.erase(it);
                } else {
                    ++it;
                }
            }
            while (!stop && !queue.empty() && (int)(active.size() + admit.size()) < max_slots) {
                Request* r = reqs[queue.front()].get();
                if (used + r->bytes > budget) break;
                queue.pop_front();
                used += r->bytes;
                r->state = RState::Running;
                admit.push_back(r);
            }
            if (active.empty() && admit.empty() && dropped.empty() && spill.empty() && fifo.empty()) {
                if (stop) break;
                cv_work.wait(lk);
                continue;
            }
        }
        for (Request* r : spill) {
            const vp_plan* p = r->plan;
            vp_status ss = VP_OK;
            try {
                const size_t rn = (size_t)p->T * p->n * p->n;
                r->h_vol.resize(p->voxels());
                r->h_proj.resize(rn);
                r->h_water.resize(rn);
                r->h_fat.resize(rn);
            } catch (const std::bad_alloc&) {
                ss = fail(VP_ERR_NOMEM, "server: out of host memory for results");
            }
            if (ss == VP_OK)
                ss = session_read(r->session.get(), r->h_vol.data(), r->h_proj.data(), r->h_water.data(),
                                  r->h_fat.data());
            r->session.reset();
            std::lock_guard<std::mutex> lk(mu);
            used -= r->bytes;
            if (r->status == VP_OK) r->status = ss;
            r->state = RState::Done;
            cv_done.notify_all();
        }
        for (Request* r : dropped) {
            r->release_events();
            r->session.reset();
            mark_done(r, VP_ERR_CANCELLED, false);
        }
        // newly admitted requests: state uploaded on their own streams, not waited for
        for (Request* r : admit) {
            vp_session* s = nullptr;
            vp_status as = session_alloc(r->plan, &r->opts, r->kspace.data(), nullptr, nullptr, &s, nullptr, false);
            if (as == VP_OK) {
                r->session.reset(s);
                as = r->make_events();
            }
            if (as != VP_OK) {
                r->session.reset();
                r->release_events();
                mark_done(r, as, false);
                continue;
            }
            active.push_back(r);
        }
        // keep up to kDepth super-steps enqueued per resident request, each on the
        // request's own stream (step graph replays); the last one carries the objective
        int feeding = 0;
        uint64_t feeding_vox = 0;
        for (Request* r : active) {
            // only requests with work left to enqueue count: the next one starts while
            // the previous one's last super-steps still run
            if (r->cancel || r->final_sent) continue;
            if (feeding > 0 && (feeding >= kStepping || feeding_vox >= kFillVoxels)) break;
            ++feeding;
            feeding_vox += r->plan->voxels();
            while (!r->cancel && r->inflight < kDepth && (r->queued < r->opts.n_steps || !r->final_sent)) {
                vp_session* s = r->session.get();
                const int64_t k = std::min<int64_t>(kSuperSteps, r->opts.n_steps - r->queued);
                vp_status st = k > 0 ? session_run(s, (int32_t)k, 1) : VP_OK;
                r->queued += k;
                const bool final = r->queued >= r->opts.n_steps;
                if (st == VP_OK && final) st = session_objective_enqueue(s, s->stream);
                hipEvent_t ev = r->ev[r->evi++ % kDepth];
                if (st == VP_OK) st = hip_status(hipEventRecord(ev, s->stream), "server event");
                fifo.push_back(Inflight{r, ev, final, st});
                r->inflight++;
                if (final) r->final_sent = true;
            }
        }
        if (fifo.empty()) continue;
        // the oldest enqueued super-step
        Inflight it = fifo.front();
        fifo.pop_front();
        Request* r = it.r;
        vp_status st = it.st;
        if (st == VP_OK) st = hip_status(hipEventSynchronize(it.ev), "server super-step");
        r->inflight--;
        // the initial upload precedes every enqueued super-step on the request's stream
        if (!r->kspace.empty() && st == VP_OK) std::vector<vp_c64>().swap(r->kspace);
        if (st != VP_OK && !r->failed) {
            r->failed = true;
            r->cancel = true;  // stop feeding; leaves when drained
            r->fail_status = st;
        }
        if (it.final || (r->failed && r->inflight == 0)) {
            if (r->inflight == 0 || !r->failed) {
                double obj = 0.0;
                vp_status fs = r->failed ? r->fail_status : session_objective_finish(r->session.get(), &obj, nullptr);
                r->final_loss = obj;
                r->steps_done = r->session->steps_done;
                if (r->failed) r->session.reset();
                r->release_events();
                active.erase(std::find(active.begin(), active.end(), r));
                mark_done(r, fs, !r->failed);
            }
        }
    }
    // shutdown: wait for enqueued work, then cancel everything still queued or running
    for (Inflight& it : fifo) (void)hipEventSynchronize(it.ev);
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active) {
        r->release_events();
        r->session.reset();
        used -= r->bytes;
        r->status = VP_ERR_CANCELLED;
        r->state = RState::Done;
    }
    for (uint64_t id : queue) {
        reqs[id]->status = VP_ERR_CANCELLED;
        reqs[id]->state = RState::Done;
    }
    queue.clear();
    cv_done.notify_all();
}

extern "C" vp_status vp_server_create(int32_t device, uint64_t hbm_budget, int32_t max_slots, vp_server** out) {
    clear_error();
    if (!out || max_slots < 1 || hbm_budget == 0) return fail(VP_ERR_ARG, "vp_server_create: bad argument");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return fail(VP_ERR_DEVICE, "vp_server_create: no device %d", device);
    std::unique_ptr<vp_server> s(new (std::nothrow) vp_server());
    if (!s) return fail(VP_ERR_NOMEM, "vp_server_create: out of host memory");
    s->device = device;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    try {
        s->worker = std::thread([p = s.get()] { p->run(); });
    } catch (...) {
        return fail(VP_ERR_STATE, "vp_server_create: cannot start the worker thread");
    }
    *out = s.release();
    return VP_OK;
}

extern "C" vp_status vp_server_submit(vp_server* s, const vp_plan* p, const vp_options* o, const vp_c64* kspace,
                                      uint64_t* request_id) {
    clear_error();
    if (!s || !p || !o || !kspace || !request_id) return fail(VP_ERR_ARG, "vp_server_submit: NULL argument");
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    const size_t nk = p->blade_px();
    for (size_t i = 0; i < nk; ++i)
        if (!std::isfinite(kspace[i].re) || !std::isfinite(kspace[i].im))
            return fail(VP_ERR_NONFINITE, "vp_server_submit: kspace holds NaN or Inf");
    uint64_t bytes = 0;
    st = vp_plan_device_bytes(p, o, &bytes);
    if (st != VP_OK) return st;
    if (bytes > s->budget)
        return fail(VP_ERR_BUDGET, "vp_server_submit: request needs %llu bytes, budget is %llu",
                    (unsigned long long)bytes, (unsigned long long)s->budget);
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return fail(VP_ERR_NOMEM, "vp_server_submit: out of host memory");
    try {
        r->kspace.assign(kspace, kspace + nk);
    } catch (const std::bad_alloc&) {
        return fail(VP_ERR_NOMEM, "vp_server_submit: out of host memory");
    }
    r->plan = p;
    r->opts = *o;
    r->opts.device = s->device;
    r->bytes = bytes;
    r->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(VP_ERR_STATE, "vp_server_submit: server is shutting down");
    r->id = s->next_id++;
    *request_id = r->id;
    if (!s->any_submit) {
        s->any_submit = true;
        s->t_first_submit = r->t_submit;
    }
    s->queue.push_back(r->id);
    s->reqs.emplace(r->id, std::move(r));
    s->cv_work.notify_one();
    return VP_OK;
}

extern "C" vp_status vp_server_wait(vp_server* s, uint64_t id, int64_t timeout_us, vp_result* result) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second->state == RState::Collecting)
        return fail(VP_ERR_NOT_FOUND, "vp_server_wait: unknown request %llu", (unsigned long long)id);
    Request* r = it->second.get();
    auto done = [r] { return r->state == RState::Done; };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return fail(VP_ERR_TIMEOUT, "vp_server_wait: request %llu still running", (unsigned long long)id);
    }
    r->state = RState::Collecting;
    std::unique_ptr<vp_session> sess = std::move(r->session);
    vp_status st = r->status;
    lk.unlock();
    // device -> caller buffers on this thread (the request's own stream), then release
    if (sess && result && st == VP_OK)
        st = session_read(sess.get(), result->volume_out, result->proj_out, result->water_out, result->fat_out);
    if (!sess && result && st == VP_OK && !r->h_vol.empty()) {
        auto copy = [](vp_c64* dst, const std::vector<vp_c64>& src) {
            if (dst) std::copy(src.begin(), src.end(), dst);
        };
        copy(result->volume_out, r->h_vol);
        copy(result->proj_out, r->h_proj);
        copy(result->water_out, r->h_water);
        copy(result->fat_out, r->h_fat);
    }
    const bool held = (bool)sess;
    sess.reset();
    lk.lock();
    if (result) {
        result->final_loss = r->final_loss;
        result->steps_done = r->steps_done;
        result->status = st;
    }
    if (held) s->used -= r->bytes;
    s->reqs.erase(id);
    s->cv_work.notify_one();
    if (st != VP_OK)
        return fail(st, "vp_server_wait: request %llu failed (%s)", (unsigned long long)id, vp_status_string(st));
    return VP_OK;
}

extern "C" vp_status vp_server_poll(vp_server* s, uint64_t id, int32_t* done) {
    clear_error();
    if (!s || !done) return fail(VP_ERR_ARG, "vp_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(VP_ERR_NOT_FOUND, "vp_server_poll: unknown request");
    *done = it->second->state == RState::Done || it->second->state == RState::Collecting;
    return VP_OK;
}

extern "C" vp_status vp_server_cancel(vp_server* s, uint64_t id) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_server_cancel: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(VP_ERR_NOT_FOUND, "vp_server_cancel: unknown request");
    Request* r = it->second.get();
    if (r->state == RState::Queued) {
        s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), id), s->queue.end());
        r->status = VP_ERR_CANCELLED;
        r->state = RState::Done;
        r->t_done = Clock::now();
        s->cv_done.notify_all();
    } else if (r->state == RState::Running) {
        r->cancel = true;
        s->cv_work.notify_one();
    }
    return VP_OK;
}

extern "C" vp_status vp_server_stats(vp_server* s, double* p50_us, double* p99_us, double* throughput_rps,
                                     int64_t* completed) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_server_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies_us;
    std::sort(l.begin(), l.end());
    auto pct = [&l](double q) {
        if (l.empty()) return 0.0;
        const size_t i = (size_t)std::ceil(q * (double)l.size()) - 1;
        return l[std::min(i, l.size() - 1)];
    };
    if (p50_us) *p50_us = pct(0.50);
    if (p99_us) *p99_us = pct(0.99);
    if (completed) *completed = (int64_t)l.size();
    if (throughput_rps) {
        const double span = std::chrono::duration<double>(s->t_last_done - s->t_first_submit).count();
        *throughput_rps = (l.empty() || span <= 0) ? 0.0 : (double)l.size() / span;
    }
    return VP_OK;
}

extern "C" vp_status vp_server_destroy(vp_server* s) {
    if (!s) return VP_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (auto& kv : s->reqs)
            if (kv.second->state == RState::Running) kv.second->cancel = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    delete s;
    return VP_OK;
}
