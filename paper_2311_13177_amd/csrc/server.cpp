// Reconstruction server: continuous batching of requests of mixed sizes on one device.
//
// A worker thread owns the device. Between super-steps it retires finished requests
// (objective, renders and volume copied to host, device state freed), drops cancelled
// ones and admits queued requests in arrival order while the sum of their device bytes
// stays within the budget and a slot is free. Every admitted request keeps its volume
// and optimiser state resident; a super-step advances all of them together with one
// launch per stage over the concatenated work lists (each request stops at its own
// step count). A request's arithmetic does not depend on the mix it runs in, so its
// result equals the one vp_reconstruct computes for it alone.

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

enum class RState { Queued, Running, Done };

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
    std::vector<vp_c64> vol, proj, water, fat;
    Clock::time_point t_submit, t_done;
    std::unique_ptr<vp_session> session;
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
    uint64_t used = 0;
    bool stop = false;
    std::vector<double> latencies_us;
    Clock::time_point t_first_submit{}, t_last_done{};
    bool any_submit = false;
    std::thread worker;
    void run();
};

namespace {

// Copies a finished session's results into the request (worker thread, no lock held).
void finish_request(Request* r) {
    vp_session* s = r->session.get();
    const vp_plan* p = r->plan;
    double obj = 0.0;
    vp_status st = session_objective(s, &obj, nullptr);
    r->final_loss = obj;
    try {
        r->vol.resize(p->voxels());
        const size_t rn = (size_t)p->T * p->n * p->n;
        r->proj.resize(rn);
        r->water.resize(rn);
        r->fat.resize(rn);
    } catch (const std::bad_alloc&) {
        st = fail(VP_ERR_NOMEM, "server: out of host memory for results");
    }
    if (st == VP_OK || st == VP_ERR_NONFINITE) {
        const vp_status rs = session_read(s, r->vol.data(), r->proj.data(), r->water.data(), r->fat.data());
        if (st == VP_OK) st = rs;
    }
    r->status = st;
    r->steps_done = r->opts.n_steps;
}

}  // namespace

void vp_server::run() {
    (void)hipSetDevice(device);
    SliceGroup g;
    g.device = device;
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess) g.stream = nullptr;
    std::vector<Request*> active;
    bool dirty = false;
    for (;;) {
        std::vector<Request*> admit;
        std::vector<Request*> dropped;
        {
            std::unique_lock<std::mutex> lk(mu);
            // cancelled running requests leave at this boundary
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->cancel) {
                    dropped.push_back(*it);
                    it = active.erase(it);
                    dirty = true;
                } else {
                    ++it;
                }
            }
            // admission: arrival order, memory budget, free slots
            while (!stop && !queue.empty() && (int)(active.size() + admit.size()) < max_slots) {
                Request* r = reqs[queue.front()].get();
                if (used + r->bytes > budget) break;
                queue.pop_front();
                used += r->bytes;
                r->state = RState::Running;
                admit.push_back(r);
            }
            if (active.empty() && admit.empty() && dropped.empty()) {
                if (stop) break;
                cv_work.wait(lk);
                continue;
            }
        }
        for (Request* r : dropped) {
            r->session.reset();
            std::lock_guard<std::mutex> lk(mu);
            used -= r->bytes;
            r->status = VP_ERR_CANCELLED;
            r->state = RState::Done;
            r->t_done = Clock::now();
            cv_done.notify_all();
        }
        for (Request* r : admit) {
            vp_session* s = nullptr;
            vp_status st = g.stream ? session_alloc(r->plan, &r->opts, r->kspace.data(), nullptr, g.stream, &s)
                                    : fail(VP_ERR_DEVICE, "server: no stream");
            std::vector<vp_c64>().swap(r->kspace);
            if (st != VP_OK) {
                std::lock_guard<std::mutex> lk(mu);
                used -= r->bytes;
                r->status = st;
                r->state = RState::Done;
                r->t_done = Clock::now();
                cv_done.notify_all();
                continue;
            }
            r->session.reset(s);
            if (r->opts.n_steps == 0) {
                finish_request(r);
                std::lock_guard<std::mutex> lk(mu);
                r->session.reset();
                used -= r->bytes;
                r->state = RState::Done;
                r->t_done = Clock::now();
                latencies_us.push_back(std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count());
                t_last_done = r->t_done;
                cv_done.notify_all();
                continue;
            }
            active.push_back(r);
            dirty = true;
        }
        if (active.empty()) continue;
        if (dirty) {
            std::vector<vp_session*> sess;
            std::vector<int> limits;
            for (Request* r : active) {
                sess.push_back(r->session.get());
                limits.push_back(r->opts.n_steps);
            }
            vp_status st = group_build(&g, sess, limits);
            if (st != VP_OK) {
                std::lock_guard<std::mutex> lk(mu);
                for (Request* r : active) {
                    r->session.reset();
                    used -= r->bytes;
                    r->status = st;
                    r->state = RState::Done;
                    r->t_done = Clock::now();
                }
                active.clear();
                cv_done.notify_all();
                continue;
            }
            dirty = false;
        }
        // one super-step: advance every resident request by up to kSuperSteps steps
        int64_t k = kSuperSteps;
        for (Request* r : active) k = std::min<int64_t>(k, r->opts.n_steps - r->session->steps_done);
        k = std::max<int64_t>(k, 1);
        vp_status st = group_run(&g, (int)k, false);
        if (st == VP_OK) st = hip_status(hipStreamSynchronize(g.stream), "server super-step");
        std::vector<Request*> finished;
        for (auto it = active.begin(); it != active.end();) {
            Request* r = *it;
            r->session->steps_done = std::min<int64_t>(r->opts.n_steps, r->session->steps_done + k);
            if (st != VP_OK || r->session->steps_done >= r->opts.n_steps) {
                finished.push_back(r);
                it = active.erase(it);
                dirty = true;
            } else {
                ++it;
            }
        }
        for (Request* r : finished) {
            if (st == VP_OK) finish_request(r);
            else r->status = st;
            r->session.reset();
            std::lock_guard<std::mutex> lk(mu);
            used -= r->bytes;
            r->state = RState::Done;
            r->t_done = Clock::now();
            latencies_us.push_back(std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count());
            t_last_done = r->t_done;
            cv_done.notify_all();
        }
    }
    // shutdown: everything still queued or running is cancelled
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : active) {
        r->session.reset();
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
    if (it == s->reqs.end()) return fail(VP_ERR_NOT_FOUND, "vp_server_wait: unknown request %llu", (unsigned long long)id);
    Request* r = it->second.get();
    auto done = [r] { return r->state == RState::Done; };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, done);
    } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done)) {
        return fail(VP_ERR_TIMEOUT, "vp_server_wait: request %llu still running", (unsigned long long)id);
    }
    const vp_status st = r->status;
    if (result) {
        auto copy = [](vp_c64* dst, const std::vector<vp_c64>& src) {
            if (dst && !src.empty()) std::copy(src.begin(), src.end(), dst);
        };
        copy(result->volume_out, r->vol);
        copy(result->proj_out, r->proj);
        copy(result->water_out, r->water);
        copy(result->fat_out, r->fat);
        result->final_loss = r->final_loss;
        result->steps_done = r->steps_done;
        result->status = st;
    }
    s->reqs.erase(it);
    if (st != VP_OK) return fail(st, "vp_server_wait: request %llu failed (%s)", (unsigned long long)id,
                                 vp_status_string(st));
    return VP_OK;
}

extern "C" vp_status vp_server_poll(vp_server* s, uint64_t id, int32_t* done) {
    clear_error();
    if (!s || !done) return fail(VP_ERR_ARG, "vp_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(VP_ERR_NOT_FOUND, "vp_server_poll: unknown request");
    *done = it->second->state == RState::Done;
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
    delete s;
    return VP_OK;
}
