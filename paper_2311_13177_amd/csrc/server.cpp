// Reconstruction server: continuous batching of requests of mixed sizes on one device.
//
// A worker thread owns the batched stepping. Each iteration it launches one super-step
// (up to kSuperSteps optimiser steps for every resident request, one launch per stage
// over the concatenated work lists, each request stopping at its own step count) and,
// while that runs on the device, finalises requests that completed in the previous
// super-step (objective on the request's own stream) and uploads newly admitted ones
// (admission in arrival order while the sum of device bytes stays within the budget
// and a slot is free). Requests join and leave only at super-step boundaries. A
// finished request keeps its device state until vp_server_wait copies the volume and
// renders straight into the caller's buffers on the caller's thread and releases it.
// A request's arithmetic does not depend on the mix it runs in, so its result equals
// the one vp_reconstruct computes for it alone.

#include <algorithm>
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

// Steps per super-step: requests join and leave only at super-step boundaries.
constexpr int kSuperSteps = 8;

enum class RState { Queued, Running, Done, Spilling, Collecting };

struct Request {
    uint64_t id = 0;
    const vp_plan* plan = nullptr;
    vp_options opts{};
    std::vector<vp_c64> kspace;
    uint64_t bytes = 0;
    RState state = RState::Queued;
    bool cancel = false;
    vp_status status = VP_OK;
    double final_loss = 0.0;
    int64_t steps_done = 0;
    Clock::time_point t_submit, t_done;
    std::unique_ptr<vp_session> session;
    // results moved to host when the device memory was needed before collection
    std::vector<vp_c64> h_vol, h_proj, h_water, h_fat;
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
    SliceGroup g;
    g.device = device;
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess) g.stream = nullptr;
    std::vector<Request*> active;     // resident and stepping
    std::vector<Request*> to_finish;  // stepped to completion, objective not yet computed
    bool dirty = false;
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
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel) {
                    dropped.push_back(*it);
                    it = active.erase(it);
                    dirty = true;
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
            if (active.empty() && admit.empty() && dropped.empty() && to_finish.empty() && spill.empty()) {
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
            r->session.reset();
            mark_done(r, VP_ERR_CANCELLED, false);
        }
        // launch the next super-step first, so the host work below overlaps it
        std::vector<Request*> stepping;
        int64_t k = 0;
        vp_status st = g.stream ? VP_OK : fail(VP_ERR_DEVICE, "server: no stream");
        if (!active.empty() && st == VP_OK) {
            if (dirty) {
                std::vector<vp_session*> sess;
                std::vector<int> limits;
                for (Request* r : active) {
                    sess.push_back(r->session.get());
                    limits.push_back(r->opts.n_steps);
                }
                st = group_build(&g, sess, limits);
                dirty = false;
            }
            if (st == VP_OK) {
                k = kSuperSteps;
                for (Request* r : active) k = std::min<int64_t>(k, r->opts.n_steps - r->session->steps_done);
                k = std::max<int64_t>(k, 1);
                st = group_run(&g, (int)k, false);
            }
            stepping = active;
        }
        // finalise the requests completed by the previous super-step (own streams)
        for (Request* r : to_finish) {
            double obj = 0.0;
            const vp_status fs = session_objective(r->session.get(), &obj, nullptr);
            r->final_loss = obj;
            r->steps_done = r->session->steps_done;
            mark_done(r, fs, true);
        }
        to_finish.clear();
        // upload newly admitted requests (own streams); they join the next super-step
        for (Request* r : admit) {
            vp_session* s = nullptr;
            const vp_status as = session_alloc(r->plan, &r->opts, r->kspace.data(), nullptr, nullptr, &s);
            std::vector<vp_c64>().swap(r->kspace);
            if (as != VP_OK) {
                mark_done(r, as, false);
                continue;
            }
            r->session.reset(s);
            if (r->opts.n_steps == 0) {
                to_finish.push_back(r);
                continue;
            }
            active.push_back(r);
            dirty = true;
        }
        if (stepping.empty()) continue;
        if (st == VP_OK) st = hip_status(hipStreamSynchronize(g.stream), "server super-step");
        for (Request* r : stepping) {
            r->session->steps_done = std::min<int64_t>(r->opts.n_steps, r->session->steps_done + k);
            if (st != VP_OK || r->session->steps_done >= r->opts.n_steps) {
                active.erase(std::find(active.begin(), active.end(), r));
                dirty = true;
                if (st != VP_OK) {
                    r->session.reset();
                    mark_done(r, st, false);
                } else {
                    to_finish.push_back(r);
                }
            }
        }
    }
    // shutdown: everything still queued or running is cancelled
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active) {
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
    if (g.stream) (void)hipStreamDestroy(g.stream);
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
