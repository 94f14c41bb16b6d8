// Batched reconstruction: many independent slices of different sizes advance together,
// one launch per stage over the concatenated work lists of every slice, with the whole
// step captured once in a HIP graph and replayed. Each slice keeps its own device
// step counter and stops at its own step count; its arithmetic is the same as alone.
// vp_batch keeps such a group resident (create, step, stage times, read, destroy);
// vp_batch_reconstruct is one pass through it.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <new>
#include <vector>

#include "plan.h"
#include "runtime.h"

namespace vp {

SliceGroup::~SliceGroup() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_descs) (void)hipFree(d_descs);
    if (d_tasks) (void)hipFree(d_tasks);
}

void SliceGroup::drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
}

// One tile shape for a whole group (the kernels take it as template parameters): the
// shape every session already uses if they agree, else the largest slice's shape when it
// fits every slice, else that shape with two-row tiles, which always fits.
static Tiles group_tiles(const std::vector<vp_session*>& sessions) {
    const vp_session* big = sessions[0];
    bool same = true;
    for (const vp_session* s : sessions) {
        same = same && s->layout->tiles == sessions[0]->layout->tiles;
        if (s->plan->voxels() > big->plan->voxels()) big = s;
    }
    Tiles t = big->layout->tiles;
    if (same) return t;
    for (const vp_session* s : sessions) {
        const Layout* L = nullptr;
        if (plan_layout(s->plan, t, &L) != VP_OK) {
            clear_error();
            t.proj_rows = 2;
            t.gath_rows = 2;
            t.gath_res = 0;
            break;
        }
    }
    return t;
}

// Builds descriptors and concatenated work lists for `sessions` (slice i = sessions[i]).
vp_status group_build(SliceGroup* g, const std::vector<vp_session*>& sessions, const std::vector<int>& limits) {
    g->drop_graph();
    const int ns = (int)sessions.size();
    std::vector<SliceDesc>& descs = g->h_descs;
    descs.assign(ns, SliceDesc{});
    std::vector<Task> proj, rows, cols, gath, vox, render, upd;
    StageLists L;
    if (ns) L.tiles = group_tiles(sessions);
    L.fft_n = ns ? sessions[0]->plan->n : 0;
    for (const vp_session* s : sessions)
        if (s->plan->n != L.fft_n) L.fft_n = 0;
    for (int i = 0; i < ns; ++i) {
        const vp_plan* p = sessions[i]->plan;
        const Layout* lay = nullptr;
        const DeviceLayout* dl = nullptr;
        vp_status st = plan_layout(p, L.tiles, &lay);
        if (st == VP_OK) st = device_layout(p, sessions[i]->tabs, lay, &dl);
        if (st != VP_OK) return st;
        if (L.tiles.upd_sc && (st = session_ensure_grad(sessions[i])) != VP_OK) return st;
        descs[i] = sessions[i]->desc;
        descs[i].groups = dl->groups;
        descs[i].step_limit = limits[i];
        auto add = [i](std::vector<Task>& dst, const std::vector<Task>& src) {
            for (Task t : src) {
                t.slice = i;
                dst.push_back(t);
            }
        };
        add(proj, lay->t_proj);
        add(rows, p->t_rows);
        add(cols, p->t_cols);
        add(gath, lay->t_gath);
        add(upd, lay->t_upd);
        add(vox, p->t_vox);
        add(render, p->t_render);
        L.re_proj = std::max(L.re_proj, lay->re_proj);
        L.lds_rows = std::max(L.lds_rows, p->lds_rows);
        L.lds_cols = std::max(L.lds_cols, p->lds_cols);
        L.re_gath = std::max(L.re_gath, lay->re_gath);
        L.lds_res = std::max(L.lds_res, lay->lds_res);
    }
    std::vector<Task>& all = g->h_tasks;
    all.clear();
    size_t off[7];
    const std::vector<Task>* parts[7] = {&proj, &rows, &cols, &gath, &vox, &render, &upd};
    for (int k = 0; k < 7; ++k) {
        off[k] = all.size();
        all.insert(all.end(), parts[k]->begin(), parts[k]->end());
    }
    hipError_t e = hipSuccess;
    // device buffers only grow (a reallocation waits for the stream to finish the old one)
    if (descs.size() > g->cap_descs || all.size() > g->cap_tasks) {
        e = hipStreamSynchronize(g->stream);
        if (e == hipSuccess && descs.size() > g->cap_descs) {
            if (g->d_descs) (void)hipFree(g->d_descs);
            g->d_descs = nullptr;
            g->cap_descs = 0;
            const size_t cap = std::max<size_t>(8, 2 * descs.size());
            e = hipMalloc((void**)&g->d_descs, cap * sizeof(SliceDesc));
            if (e == hipSuccess) g->cap_descs = cap;
        }
        if (e == hipSuccess && all.size() > g->cap_tasks) {
            if (g->d_tasks) (void)hipFree(g->d_tasks);
            g->d_tasks = nullptr;
            g->cap_tasks = 0;
            const size_t cap = std::max<size_t>(1024, all.size() + all.size() / 2);
            e = hipMalloc((void**)&g->d_tasks, cap * sizeof(Task));
            if (e == hipSuccess) g->cap_tasks = cap;
        }
    }
    if (e == hipSuccess && ns)
        e = hipMemcpyAsync(g->d_descs, descs.data(), descs.size() * sizeof(SliceDesc), hipMemcpyHostToDevice,
                           g->stream);
    if (e == hipSuccess && !all.empty())
        e = hipMemcpyAsync(g->d_tasks, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice, g->stream);
    if (e != hipSuccess) return hip_status(e, "slice group upload");
    L.proj = g->d_tasks + off[0]; L.n_proj = (int)proj.size();
    L.rows = g->d_tasks + off[1]; L.n_rows = (int)rows.size();
    L.cols = g->d_tasks + off[2]; L.n_cols = (int)cols.size();
    L.gath = g->d_tasks + off[3]; L.n_gath = (int)gath.size();
    L.vox = g->d_tasks + off[4]; L.n_vox = (int)vox.size();
    L.render = g->d_tasks + off[5]; L.n_render = (int)render.size();
    L.upd = g->d_tasks + off[6]; L.n_upd = (int)upd.size();
    L.n_slices = ns;
    L.epi = EPI_ADAM_TV;
    uint64_t nvox = 0;
    for (const vp_session* se : sessions) {
        if (se->lists.epi != EPI_ADAM_TV) L.epi = EPI_GENERIC;
        nvox += se->plan->voxels();
    }
    L.stream = stream_for(nvox, VP_OPT_ADAM);
    g->lists = L;
    return VP_OK;
}

// Enqueues n_steps steps of every slice in the group; use_graph captures one step once.
vp_status group_run(SliceGroup* g, int n_steps, bool use_graph) {
    KArgs a{};
    a.descs = g->d_descs;
    hipError_t e;
    if (use_graph) {
        if (!g->gexec) {
            e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_status(e, "hipStreamBeginCapture");
            hipError_t le = hipSuccess;
            launch_step(a, g->lists, g->stream, &le);
            e = hipStreamEndCapture(g->stream, &g->graph);
            if (le != hipSuccess) return hip_status(le, "batched step capture");
            if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&g->gexec, g->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return hip_status(e, "hipGraphInstantiate");
        }
        for (int i = 0; i < n_steps; ++i)
            if ((e = hipGraphLaunch(g->gexec, g->stream)) != hipSuccess) return hip_status(e, "hipGraphLaunch");
    } else {
        for (int i = 0; i < n_steps; ++i) {
            launch_step(a, g->lists, g->stream, &e);
            if (e != hipSuccess) return hip_status(e, "batched step launch");
        }
    }
    return VP_OK;
}

}  // namespace vp

using namespace vp;

// A resident batch: the slices' sessions on one stream, grouped for batched launches.
struct vp_batch {
    vp::SliceGroup g;
    std::vector<std::unique_ptr<vp_session>> owned;
    std::vector<vp_session*> sessions;   // admitted slices, in input order
    std::vector<int> limits;             // their step counts
    std::vector<int> slot_of;            // input index -> slot in sessions (-1: failed)
    std::vector<vp_status> status;       // per input slice
    int max_steps = 0;
    int64_t steps_run = 0;               // batched steps enqueued so far
    ~vp_batch() {
        if (g.stream) {
            (void)hipSetDevice(g.device);
            (void)hipStreamSynchronize(g.stream);
        }
        owned.clear();
        g.drop_graph();
        if (g.stream) (void)hipStreamDestroy(g.stream);
        g.stream = nullptr;
    }
};

extern "C" vp_status vp_batch_create(int32_t n, const vp_plan* const* plans, const vp_options* const* opts,
                                     const vp_c64* const* kspace, vp_batch** out) {
    clear_error();
    if (!out || n < 1 || !plans || !opts || !kspace) return fail(VP_ERR_ARG, "vp_batch_create: bad argument");
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !opts[i] || !kspace[i]) return fail(VP_ERR_ARG, "vp_batch_create: NULL entry %d", i);
    const int device = opts[0]->device;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    std::unique_ptr<vp_batch> b(new (std::nothrow) vp_batch());
    if (!b) return fail(VP_ERR_NOMEM, "vp_batch_create: out of host memory");
    b->g.device = device;
    e = hipStreamCreateWithFlags(&b->g.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        b->g.stream = nullptr;
        return hip_status(e, "hipStreamCreate");
    }
    b->slot_of.assign(n, -1);
    b->status.assign(n, VP_OK);
    // One tile shape serves the whole batch: when any slice asks for tuning, the
    // largest slice is tuned (once per plan sizes) and every slice whose regions fit
    // takes its shape.
    bool tune = false;
    int big = 0;
    for (int i = 0; i < n; ++i) {
        tune = tune || opts[i]->autotune != 0;
        if (plans[i]->voxels() > plans[big]->voxels()) big = i;
    }
    Tiles shape{};
    bool have_shape = false;
    if (tune) {
        vp_options ob = *opts[big];
        ob.device = device;
        ob.autotune = 1;
        have_shape = check_options(plans[big], &ob) == VP_OK && tiles_for(plans[big], &ob, &shape) == VP_OK;
        if (!have_shape) clear_error();
    }
    vp_status first_err = VP_OK;
    for (int i = 0; i < n; ++i) {
        vp_options o = *opts[i];
        o.device = device;
        o.autotune = 0;
        const vp_tiles& ot = o.tiles;
        const Layout* lay = nullptr;
        const bool unset = !ot.proj_rows && !ot.proj_parts && !ot.gath_rows && !ot.gath_bins && !ot.upd_bins &&
                           !ot.gath_waves && !ot.proj_waves && !ot.gath_resident;
        if (have_shape && unset) {
            if (plan_layout(plans[i], shape, &lay) == VP_OK)
                o.tiles = vp_tiles{shape.proj_rows, shape.proj_gw, shape.gath_rows, shape.gath_sc,
                                   shape.upd_sc, shape.gath_w, shape.proj_w, shape.gath_res};
            else
                clear_error();
        }
        vp_session* s = nullptr;
        const vp_status st = session_alloc(plans[i], &o, kspace[i], nullptr, b->g.stream, &s);
        b->status[i] = st;
        if (st != VP_OK) {
            if (first_err == VP_OK) first_err = st;
            continue;
        }
        b->slot_of[i] = (int)b->sessions.size();
        b->owned.emplace_back(s);
        b->sessions.push_back(s);
        b->limits.push_back(o.n_steps);
        b->max_steps = std::max(b->max_steps, o.n_steps);
    }
    if (b->sessions.empty()) return first_err;
    const vp_status st = group_build(&b->g, b->sessions, b->limits);
    if (st != VP_OK) return st;
    *out = b.release();
    return first_err == VP_OK ? VP_OK : first_err;
}

extern "C" vp_status vp_batch_step(vp_batch* b, int32_t n_steps, int32_t use_graph) {
    clear_error();
    if (!b || n_steps < 0) return fail(VP_ERR_ARG, "vp_batch_step: bad argument");
    hipError_t e = hipSetDevice(b->g.device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    vp_status st = group_run(&b->g, n_steps, use_graph != 0);
    if (st == VP_OK) st = hip_status(hipStreamSynchronize(b->g.stream), "batched steps");
    if (st != VP_OK) return st;
    b->steps_run += n_steps;
    for (size_t k = 0; k < b->sessions.size(); ++k)
        b->sessions[k]->steps_done = std::min<int64_t>(b->limits[k], b->steps_run);
    return VP_OK;
}

extern "C" vp_status vp_batch_stage_times(vp_batch* b, int32_t n_steps, double* stage_ms) {
    clear_error();
    if (!b || !stage_ms || n_steps < 1 || n_steps > 100000) return fail(VP_ERR_ARG, "vp_batch_stage_times: bad argument");
    hipError_t e = hipSetDevice(b->g.device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    const int ne = (kStages + 1) * n_steps;
    std::vector<hipEvent_t> ev(ne, nullptr);
    vp_status st = VP_OK;
    for (int i = 0; i < ne && st == VP_OK; ++i) st = hip_status(hipEventCreate(&ev[i]), "hipEventCreate");
    KArgs a{};
    a.descs = b->g.d_descs;
    for (int k = 0; k < n_steps && st == VP_OK; ++k) {
        launch_step(a, b->g.lists, b->g.stream, &e, &ev[(size_t)k * (kStages + 1)]);
        st = hip_status(e, "stage-timed batched step");
    }
    if (st == VP_OK) st = hip_status(hipStreamSynchronize(b->g.stream), "stage-timed batched steps");
    if (st == VP_OK) {
        b->steps_run += n_steps;
        for (size_t k = 0; k < b->sessions.size(); ++k)
            b->sessions[k]->steps_done = std::min<int64_t>(b->limits[k], b->steps_run);
    }
    for (int j = 0; j < kStages; ++j) stage_ms[j] = 0.0;
    for (int k = 0; k < n_steps && st == VP_OK; ++k)
        for (int j = 0; j < kStages && st == VP_OK; ++j) {
            float ms = 0.f;
            hipEvent_t* bv = &ev[(size_t)k * (kStages + 1)];
            st = hip_status(hipEventElapsedTime(&ms, bv[j], bv[j + 1]), "hipEventElapsedTime");
            stage_ms[j] += ms / n_steps;
        }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    return st;
}

extern "C" vp_status vp_batch_read(vp_batch* b, int32_t i, vp_result* r) {
    clear_error();
    if (!b || !r || i < 0 || i >= (int)b->slot_of.size()) return fail(VP_ERR_ARG, "vp_batch_read: bad argument");
    if (b->slot_of[i] < 0) {
        r->status = b->status[i];
        r->steps_done = 0;
        r->final_loss = 0.0;
        return r->status;
    }
    hipError_t e = hipSetDevice(b->g.device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    vp_session* s = b->sessions[b->slot_of[i]];
    double obj = 0.0;
    vp_status st = session_objective(s, &obj, nullptr);
    const vp_status rs = session_read(s, r->volume_out, r->proj_out, r->water_out, r->fat_out);
    if (st == VP_OK) st = rs;
    r->final_loss = obj;
    r->steps_done = s->steps_done;
    r->status = st;
    return st;
}

extern "C" vp_status vp_batch_destroy(vp_batch* b) {
    delete b;
    return VP_OK;
}

extern "C" vp_status vp_batch_reconstruct(int32_t n, const vp_plan* const* plans, const vp_options* const* opts,
                                          const vp_c64* const* kspace, vp_result* const* results) {
    clear_error();
    if (n < 0 || (n > 0 && (!plans || !opts || !kspace || !results)))
        return fail(VP_ERR_ARG, "vp_batch_reconstruct: bad argument");
    if (n == 0) return VP_OK;
    for (int i = 0; i < n; ++i)
        if (!plans[i] || !opts[i] || !kspace[i] || !results[i])
            return fail(VP_ERR_ARG, "vp_batch_reconstruct: NULL entry %d", i);
    for (int i = 0; i < n; ++i) {
        results[i]->status = VP_OK;
        results[i]->steps_done = 0;
        results[i]->final_loss = 0.0;
    }
    vp_batch* raw = nullptr;
    const vp_status cst = vp_batch_create(n, plans, opts, kspace, &raw);
    if (!raw) {
        // no slice could be set up (or the group failed): report per-slice allocation errors
        for (int i = 0; i < n; ++i) results[i]->status = cst;
        return cst;
    }
    std::unique_ptr<vp_batch> b(raw);
    vp_status first_err = cst;
    vp_status st = vp_batch_step(b.get(), b->max_steps, 1);
    if (st != VP_OK) return st;
    for (int i = 0; i < n; ++i) {
        st = vp_batch_read(b.get(), i, results[i]);
        if (st != VP_OK && first_err == VP_OK) first_err = st;
    }
    return first_err;
}
