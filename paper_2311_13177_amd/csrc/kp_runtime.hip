// Host side of the K-Planes dynamic model (Section 4.1): model validation and layout,
// interpolation tables, the gradient and decode operators, and resident fits whose
// step is captured in a HIP graph. The dense per-blade volumes go through the lifted
// projection, blur and adjoint kernels of a per-blade plan (one knot per blade).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <memory>
#include <vector>

#include "kplanes.h"
#include "plan.h"
#include "runtime.h"
#include "vp.h"

namespace vp {
namespace {

vp_status check_model(const vp_plan* p, const vp_kplanes* m) {
    if (!p || !m) return fail(VP_ERR_ARG, "K-Planes: NULL plan or model");
    if (!kp_features_ok(m->features)) return fail(VP_ERR_ARG, "K-Planes: features must be 1, 2, 4, 8 or 16");
    if (m->time_res < 1 || m->time_res > 4096) return fail(VP_ERR_ARG, "K-Planes: time_res outside [1, 4096]");
    if (m->n_scales < 1 || m->n_scales > VP_KP_MAX_SCALES)
        return fail(VP_ERR_ARG, "K-Planes: n_scales outside [1, %d]", VP_KP_MAX_SCALES);
    for (int c = 0; c < m->n_scales; ++c)
        if (m->spatial_res[c] < 1 || m->spatial_res[c] > p->n)
            return fail(VP_ERR_ARG, "K-Planes: spatial_res[%d] outside [1, n]", c);
    if (!std::isfinite(m->tv_weight) || !std::isfinite(m->smooth_weight) || !std::isfinite(m->sparse_weight))
        return fail(VP_ERR_ARG, "K-Planes: regulariser weights must be finite");
    if (!(m->eps > 0.f) || !std::isfinite(m->eps)) return fail(VP_ERR_ARG, "K-Planes: eps must be > 0");
    return VP_OK;
}

// Sizes, offsets and interpolation tables of a model at a list of times (host side).
struct KPTables {
    KPDesc d{};
    std::vector<int> nd0, tr_ptr, tr_smp, tk, tt_ptr, tt_b;
    std::vector<float> ndw, tr_w, ta, tt_w;
};

void build_tables(const vp_plan* p, const vp_kplanes* m, const double* times, int nt, KPTables* t) {
    KPDesc& d = t->d;
    d = KPDesc{};
    d.n = p->n; d.S = p->S; d.B = nt; d.F = m->features; d.Rt = m->time_res; d.ns = m->n_scales;
    long long off = 0;
    for (int c = 0; c < d.ns; ++c) {
        const long long R = m->spatial_res[c];
        d.R[c] = (int)R;
        const long long sz[KP_PLANES] = {R * R, d.S * R, d.S * R, d.Rt * R, d.Rt * R, (long long)d.Rt * d.S};
        for (int g = 0; g < KP_PLANES; ++g) {
            d.off[c][g] = off;
            off += sz[g] * d.F;
        }
    }
    d.a_off = off;
    d.n_params = off + d.F;
    const int n = d.n;
    // spatial nodes per scale and their transposes (samples ascending per node)
    t->nd0.assign((size_t)d.ns * n, 0);
    t->ndw.assign((size_t)d.ns * n, 0.f);
    t->tr_ptr.assign((size_t)d.ns * (n + 1), 0);
    t->tr_smp.clear();
    t->tr_w.clear();
    for (int c = 0; c < d.ns; ++c) {
        const int R = d.R[c];
        std::vector<double> w(n, 0.0);
        for (int i = 0; i < n; ++i) {
            int i0 = 0;
            if (R > 1) {
                const double u = n > 1 ? (double)i * (R - 1) / (double)(n - 1) : 0.0;
                i0 = std::min((int)std::floor(u), R - 2);
                w[i] = u - i0;
            }
            t->nd0[(size_t)c * n + i] = i0;
            t->ndw[(size_t)c * n + i] = (float)w[i];
        }
        for (int j = 0; j < R; ++j) {
            t->tr_ptr[(size_t)c * (n + 1) + j] = (int)t->tr_smp.size();
            for (int i = 0; i < n; ++i) {
                const int i0 = t->nd0[(size_t)c * n + i];
                if (i0 == j && 1.0 - w[i] != 0.0) {
                    t->tr_smp.push_back(i);
                    t->tr_w.push_back((float)(1.0 - w[i]));
                }
                if (R > 1 && i0 + 1 == j && w[i] != 0.0) {
                    t->tr_smp.push_back(i);
                    t->tr_w.push_back((float)w[i]);
                }
            }
        }
        for (int j = R; j <= n; ++j) t->tr_ptr[(size_t)c * (n + 1) + j] = (int)t->tr_smp.size();
    }
    // time nodes per time and their transposes (times ascending per node)
    const int Rt = d.Rt;
    t->tk.assign(nt, 0);
    t->ta.assign(nt, 0.f);
    std::vector<double> a(nt, 0.0);
    for (int b = 0; b < nt; ++b) {
        if (Rt > 1) {
            const double u = times[b] * (Rt - 1);
            const int k = std::min((int)std::floor(u), Rt - 2);
            t->tk[b] = k;
            a[b] = u - k;
            t->ta[b] = (float)a[b];
        }
    }
    t->tt_ptr.assign(Rt + 1, 0);
    t->tt_b.clear();
    t->tt_w.clear();
    for (int k = 0; k < Rt; ++k) {
        t->tt_ptr[k] = (int)t->tt_b.size();
        for (int b = 0; b < nt; ++b) {
            if (t->tk[b] == k && 1.0 - a[b] != 0.0) {
                t->tt_b.push_back(b);
                t->tt_w.push_back((float)(1.0 - a[b]));
            }
            if (Rt > 1 && t->tk[b] + 1 == k && a[b] != 0.0) {
                t->tt_b.push_back(b);
                t->tt_w.push_back((float)a[b]);
            }
        }
    }
    t->tt_ptr[Rt] = (int)t->tt_b.size();
    // keep the CSR arrays non-empty so every device copy has a valid source
    if (t->tr_smp.empty()) { t->tr_smp.push_back(0); t->tr_w.push_back(0.f); }
    if (t->tt_b.empty()) { t->tt_b.push_back(0); t->tt_w.push_back(0.f); }
}

// Device allocations of one model evaluation or fit, freed together.
struct DevArena {
    std::vector<void*> ptrs;
    ~DevArena() {
        for (void* q : ptrs) (void)hipFree(q);
    }
    template <class T>
    hipError_t alloc(T** out, size_t count) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return e;
        ptrs.push_back(q);
        *out = (T*)q;
        return hipSuccess;
    }
    template <class T>
    hipError_t upload(T** out, const std::vector<T>& v, hipStream_t s) {
        hipError_t e = alloc(out, v.size());
        if (e == hipSuccess && !v.empty())
            e = hipMemcpyAsync(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
        return e;
    }
};

// Tables and factor buffers on the device; with_grad also the gradient buffers.
hipError_t kp_device(KPTables* t, DevArena* ar, bool with_grad, hipStream_t s) {
    KPDesc& d = t->d;
    hipError_t e = hipSuccess;
    auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ok(ar->upload((int**)&d.nd0, t->nd0, s));
    ok(ar->upload((float**)&d.ndw, t->ndw, s));
    ok(ar->upload((int**)&d.tr_ptr, t->tr_ptr, s));
    ok(ar->upload((int**)&d.tr_smp, t->tr_smp, s));
    ok(ar->upload((float**)&d.tr_w, t->tr_w, s));
    ok(ar->upload((int**)&d.tk, t->tk, s));
    ok(ar->upload((float**)&d.ta, t->ta, s));
    ok(ar->upload((int**)&d.tt_ptr, t->tt_ptr, s));
    ok(ar->upload((int**)&d.tt_b, t->tt_b, s));
    ok(ar->upload((float**)&d.tt_w, t->tt_w, s));
    const size_t ns = d.ns, S = d.S, n = d.n, B = d.B, F = d.F;
    ok(ar->alloc(&d.Xs, ns * S * n * F));
    ok(ar->alloc(&d.Ys, ns * S * n * F));
    ok(ar->alloc(&d.qx, ns * B * n * F));
    ok(ar->alloc(&d.qy, ns * B * n * F));
    ok(ar->alloc(&d.qs, ns * B * S * F));
    ok(ar->alloc(&d.Z, ns * n * n * F));
    ok(ar->alloc(&d.XA, ns * B * S * n * F));
    ok(ar->alloc(&d.Yf, ns * B * S * n * F));
    if (with_grad) {
        ok(ar->alloc(&d.gZ, ns * n * n * F));
        // enough (b, s) chunks for about 4096 wave tasks (two rows by 64 columns) in the
        // xy-gradient pass
        d.zchunks = (int)std::max<size_t>(1, std::min<size_t>(B * S, (524288 + n * n - 1) / (n * n)));
        ok(ar->alloc(&d.zpart, (size_t)d.zchunks * ns * n * n * F));
        ok(ar->alloc(&d.gXA, 2 * ns * B * S * n * F));
        ok(ar->alloc(&d.gY, ns * B * S * n * F));
        ok(ar->alloc(&d.gXs, ns * S * n * F));
        ok(ar->alloc(&d.gYs, ns * S * n * F));
        ok(ar->alloc(&d.gqx, ns * B * n * F));
        ok(ar->alloc(&d.gqy, ns * B * n * F));
        ok(ar->alloc(&d.gqs, ns * B * S * F));
        ok(ar->alloc(&d.h, ns * B * S * F));
        ok(ar->alloc(&d.ga, F));
        ok(ar->alloc(&d.rpart, (size_t)kp_reg_blocks(d)));
    }
    return e;
}

void set_regs(KPDesc* d, const vp_kplanes* m) {
    d->tv_w = m->tv_weight;
    d->smooth_w = m->smooth_weight;
    d->sparse_w = m->sparse_weight;
    d->eps2 = std::max(m->eps * m->eps, FLT_MIN);
}

// The dense stages of a step on the per-blade plan q: projection of every blade's own
// volume, DFT passes with mask, residual and loss partials, inverse passes and the
// transposed projection into G (stored, not accumulated).
struct DenseStep {
    const vp_plan* q = nullptr;
    DeviceTables* tabs = nullptr;
    const Layout* lay = nullptr;
    const DeviceLayout* dl = nullptr;
    StageLists L{};
    KArgs a{};
};

// The per-blade plan's tile shape: the one recorded by the autotuner for its sizes, else
// (opts asking for it) tuned now, else the plan's heuristic shape.
vp_status dense_setup(const vp_plan* p, DenseStep* ds, const vp_options* o = nullptr) {
    vp_status st = plan_per_blade(p, &ds->q);
    if (st == VP_OK) st = plan_tables(ds->q, &ds->tabs);
    Tiles t = ds->q->base_tiles;
    if (st == VP_OK && !tuned_tiles(ds->q, ds->tabs->device, o ? o->optimizer : VP_OPT_ADAM, &t) && o &&
        o->autotune) {
        vp_options to = *o;
        to.tiles = vp_tiles{0, 0, 0, 0, 0, 0, 0, 0};
        st = tune_plan(ds->q, &to, &t);
    }
    if (st == VP_OK) st = plan_layout(ds->q, t, &ds->lay);
    if (st == VP_OK) st = device_layout(ds->q, ds->tabs, ds->lay, &ds->dl);
    if (st != VP_OK) return st;
    ds->L = plan_lists(ds->q, ds->tabs, ds->lay, ds->dl);
    ds->a = KArgs{};
    fill_desc(ds->q, ds->tabs, ds->lay, ds->dl, &ds->a.one);
    return VP_OK;
}

hipError_t dense_forward(const DenseStep& ds, hipStream_t s) {
    KArgs a = ds.a;
    const StageLists& L = ds.L;
    hipError_t e;
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, s)) != hipSuccess) return e;
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, -1, L.fft_n, L.lds_rows, s)) != hipSuccess) return e;
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_STEP;
    return launch_cols(a, L.fft_n, L.lds_cols, s);
}

hipError_t dense_adjoint(const DenseStep& ds, hipStream_t s) {
    KArgs a = ds.a;
    const StageLists& L = ds.L;
    hipError_t e;
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, 1, L.fft_n, L.lds_rows, s)) != hipSuccess) return e;
    a.tasks = L.gath; a.ntasks = L.n_gath; a.accumulate = 0;
    return launch_gather_lists(a, GATHER_STORE, L, s);
}

double host_objective(const std::vector<float>& lp, const std::vector<double>& rp, double* data) {
    double dl = 0.0, r = 0.0;
    for (float v : lp) dl += (double)v;
    dl *= 0.5;
    for (double v : rp) r += v;
    if (data) *data = dl;
    return dl + r;
}

}  // namespace
}  // namespace vp

using namespace vp;

// ------------------------------------------------------------------ operators

extern "C" vp_status vp_kplanes_param_count(const vp_plan* p, const vp_kplanes* m, int64_t* count) {
    clear_error();
    if (!count) return fail(VP_ERR_ARG, "vp_kplanes_param_count: NULL output");
    vp_status st = check_model(p, m);
    if (st != VP_OK) return st;
    KPTables t;
    double zero = 0.0;
    build_tables(p, m, &zero, 1, &t);
    *count = t.d.n_params;
    return VP_OK;
}

extern "C" vp_status vp_kplanes_decode(const vp_plan* p, const vp_kplanes* m, const vp_c64* d_params,
                                       const double* times, int32_t n_times, vp_c64* d_vol, void* stream) {
    clear_error();
    vp_status st = check_model(p, m);
    if (st != VP_OK) return st;
    if (n_times < 0) return fail(VP_ERR_ARG, "vp_kplanes_decode: n_times < 0");
    if (n_times == 0) return VP_OK;
    if (!d_params || !times || !d_vol) return fail(VP_ERR_ARG, "vp_kplanes_decode: NULL argument");
    for (int i = 0; i < n_times; ++i)
        if (!std::isfinite(times[i]) || times[i] < 0.0 || times[i] > 1.0)
            return fail(VP_ERR_ARG, "vp_kplanes_decode: times[%d] outside [0, 1]", i);
    hipStream_t s = (hipStream_t)stream;
    KPTables t;
    build_tables(p, m, times, n_times, &t);
    DevArena ar;
    hipError_t e = kp_device(&t, &ar, false, s);
    t.d.params = (float2*)d_params;
    t.d.vol = (float2*)d_vol;
    if (e == hipSuccess) e = kp_launch_factors(t.d, s);
    if (e == hipSuccess) e = kp_launch_decode(t.d, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    return hip_status(e, "vp_kplanes_decode");
}

extern "C" vp_status vp_kplanes_gradient(const vp_plan* p, const vp_kplanes* m, const vp_c64* d_params,
                                         const vp_c64* d_kspace, vp_c64* d_grad, double* objective,
                                         double* data_term, void* stream) {
    clear_error();
    vp_status st = check_model(p, m);
    if (st != VP_OK) return st;
    if (!d_params || !d_kspace || !d_grad) return fail(VP_ERR_ARG, "vp_kplanes_gradient: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    DenseStep ds;
    if ((st = dense_setup(p, &ds)) != VP_OK) return st;
    KPTables t;
    build_tables(p, m, p->tau.data(), p->B, &t);
    set_regs(&t.d, m);
    DevArena ar;
    hipError_t e = kp_device(&t, &ar, true, s);
    const size_t nvol = (size_t)p->B * p->S * p->n * p->n;
    float2 *vol = nullptr, *G = nullptr, *work = nullptr;
    float* lp = nullptr;
    const size_t nl = loss_slots(ds.q);
    if (e == hipSuccess) e = ar.alloc(&vol, nvol);
    if (e == hipSuccess) e = ar.alloc(&G, nvol);
    if (e == hipSuccess) e = ar.alloc(&work, (size_t)ds.q->nparts * ds.q->blade_px());
    if (e == hipSuccess) e = ar.alloc(&lp, nl);
    KPDesc& d = t.d;
    d.params = (float2*)d_params;
    d.grad = (float2*)d_grad;
    d.vol = vol;
    d.G = G;
    ds.a.one.vol[0] = vol;
    ds.a.one.work = work;
    ds.a.one.y = (const float2*)d_kspace;
    ds.a.one.loss_part = lp;
    ds.a.one.grad = G;
    if (e == hipSuccess) e = kp_launch_factors(d, s);
    if (e == hipSuccess) e = kp_launch_decode(d, s);
    if (e == hipSuccess) e = dense_forward(ds, s);
    if (e == hipSuccess) e = dense_adjoint(ds, s);
    if (e == hipSuccess) e = kp_launch_back(d, s);
    if (e == hipSuccess) e = kp_launch_chain(d, s);
    if (e == hipSuccess) e = kp_launch_reg_value(d, s);
    std::vector<float> hl(nl);
    std::vector<double> hr((size_t)kp_reg_blocks(d));
    if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), lp, nl * sizeof(float), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), d.rpart, hr.size() * sizeof(double), hipMemcpyDeviceToHost, s);
    const hipError_t e2 = hipStreamSynchronize(s);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_status(e, "vp_kplanes_gradient");
    const double obj = host_objective(hl, hr, data_term);
    if (objective) *objective = obj;
    if (!std::isfinite(obj)) return fail(VP_ERR_NONFINITE, "vp_kplanes_gradient: objective is not finite");
    return VP_OK;
}

// ------------------------------------------------------------------ resident fits

struct vp_kplanes_session {
    const vp_plan* plan = nullptr;
    vp_kplanes model{};
    vp_options opts{};
    int device = -1;
    hipStream_t stream = nullptr;
    vp::KPTables tab;
    vp::DevArena ar;
    vp::DenseStep ds;
    float* loss_part = nullptr;
    int* step_dev = nullptr;
    int64_t steps_done = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    ~vp_kplanes_session() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

constexpr int kKpStages = 6;

// One fit step; with ev (kKpStages + 1 events) an event before each stage and after the last.
hipError_t kp_step(vp_kplanes_session* s, hipEvent_t* ev) {
    const KPDesc& d = s->tab.d;
    hipStream_t st = s->stream;
    hipError_t e = hipSuccess;
    auto mark = [&](int i) {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[i], st);
    };
    mark(0);
    if (e == hipSuccess) e = kp_launch_factors(d, st);
    if (e == hipSuccess) e = kp_launch_decode(d, st);
    mark(1);
    if (e == hipSuccess) e = dense_forward(s->ds, st);
    if (e == hipSuccess) e = dense_adjoint(s->ds, st);
    mark(2);
    if (e == hipSuccess) e = kp_launch_back_z(d, st);
    mark(3);
    if (e == hipSuccess) e = kp_launch_back_x(d, st);
    mark(4);
    if (e == hipSuccess) e = kp_launch_back_y(d, st);
    mark(5);
    if (e == hipSuccess) e = kp_launch_chain(d, st);
    if (e == hipSuccess) e = kp_launch_update(d, st);
    mark(6);
    return e;
}

}  // namespace

extern "C" vp_status vp_kplanes_session_create(const vp_plan* p, const vp_kplanes* m, const vp_options* o,
                                               const vp_c64* kspace, const vp_c64* init, vp_kplanes_session** out) {
    clear_error();
    if (!o || !kspace || !init || !out) return fail(VP_ERR_ARG, "vp_kplanes_session_create: NULL argument");
    vp_status st = check_model(p, m);
    if (st != VP_OK) return st;
    if ((st = check_options(p, o)) != VP_OK) return st;
    if (o->schedule != VP_SCHED_ALL_BLADES)
        return fail(VP_ERR_UNSUPPORTED, "vp_kplanes_session_create: only the all-blades schedule is supported");
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    std::unique_ptr<vp_kplanes_session> s(new (std::nothrow) vp_kplanes_session());
    if (!s) return fail(VP_ERR_NOMEM, "vp_kplanes_session_create: out of host memory");
    s->plan = p;
    s->model = *m;
    s->opts = *o;
    s->device = o->device;
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_status(e, "stream");
    if ((st = dense_setup(p, &s->ds, o)) != VP_OK) return st;
    s->ds.a.one.data_w = o->data_weight;
    build_tables(p, m, p->tau.data(), p->B, &s->tab);
    KPDesc& d = s->tab.d;
    set_regs(&d, m);
    d.optimizer = o->optimizer;
    d.lr = o->lr;
    d.beta1 = o->beta1;
    d.beta2 = o->beta2;
    d.c1 = 1.0f - o->beta1;
    d.c2 = 1.0f - o->beta2;
    d.aeps = o->adam_eps;
    d.ln_beta1 = (float)std::log((double)o->beta1);
    d.ln_beta2 = (float)std::log((double)o->beta2);
    hipStream_t ss = s->stream;
    e = kp_device(&s->tab, &s->ar, true, ss);
    const size_t np = (size_t)d.n_params;
    const size_t nvol = (size_t)p->B * p->S * p->n * p->n;
    const size_t nl = loss_slots(s->ds.q);
    float2 *params = nullptr, *grad = nullptr, *y = nullptr, *work = nullptr, *G = nullptr;
    auto ok = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    ok(s->ar.alloc(&params, np));
    ok(s->ar.alloc(&grad, np));
    ok(s->ar.alloc(&d.m, np));
    ok(s->ar.alloc(&d.v, np));
    ok(s->ar.alloc(&d.vol, nvol));
    ok(s->ar.alloc(&G, nvol));
    ok(s->ar.alloc(&y, s->ds.q->blade_px()));
    ok(s->ar.alloc(&work, (size_t)s->ds.q->nparts * s->ds.q->blade_px()));
    ok(s->ar.alloc(&s->loss_part, nl));
    ok(s->ar.alloc(&s->step_dev, 1));
    if (e != hipSuccess) return hip_status(e, "vp_kplanes_session_create");
    ok(hipMemcpyAsync(params, init, np * sizeof(float2), hipMemcpyHostToDevice, ss));
    ok(hipMemcpyAsync(y, kspace, s->ds.q->blade_px() * sizeof(float2), hipMemcpyHostToDevice, ss));
    ok(hipMemsetAsync(d.m, 0, np * sizeof(float2), ss));
    ok(hipMemsetAsync(d.v, 0, np * sizeof(float2), ss));
    ok(hipMemsetAsync(s->step_dev, 0, sizeof(int), ss));
    ok(hipStreamSynchronize(ss));
    if (e != hipSuccess) return hip_status(e, "vp_kplanes_session_create upload");
    d.params = params;
    d.grad = grad;
    d.G = G;
    d.step = s->step_dev;
    s->ds.a.one.vol[0] = d.vol;
    s->ds.a.one.work = work;
    s->ds.a.one.y = y;
    s->ds.a.one.loss_part = s->loss_part;
    s->ds.a.one.grad = G;
    *out = s.release();
    return VP_OK;
}

extern "C" vp_status vp_kplanes_session_step(vp_kplanes_session* s, int32_t n_steps, int32_t use_graph) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_kplanes_session_step: NULL session");
    if (n_steps < 0) return fail(VP_ERR_ARG, "vp_kplanes_session_step: n_steps < 0");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    if (use_graph && !s->gexec && n_steps > 0) {
        e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
        hipError_t le = hipSuccess;
        if (e == hipSuccess) le = kp_step(s, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(s->stream, &g);
        if (e == hipSuccess) e = le != hipSuccess ? le : ce;
        if (e == hipSuccess) e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_status(e, "vp_kplanes_session_step capture");
        }
        s->graph = g;
    }
    for (int i = 0; i < n_steps && e == hipSuccess; ++i)
        e = use_graph ? hipGraphLaunch(s->gexec, s->stream) : kp_step(s, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_status(e, "vp_kplanes_session_step");
    s->steps_done += n_steps;
    return VP_OK;
}

extern "C" vp_status vp_kplanes_session_read(vp_kplanes_session* s, vp_c64* params_out, int32_t n_frames,
                                             const double* frame_times, vp_c64* proj_out, vp_c64* water_out,
                                             vp_c64* fat_out, double* objective) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_kplanes_session_read: NULL session");
    if (n_frames < 0 || (n_frames > 0 && !frame_times)) return fail(VP_ERR_ARG, "vp_kplanes_session_read: frames");
    for (int i = 0; i < n_frames; ++i)
        if (!std::isfinite(frame_times[i]) || frame_times[i] < 0.0 || frame_times[i] > 1.0)
            return fail(VP_ERR_ARG, "vp_kplanes_session_read: frame_times[%d] outside [0, 1]", i);
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    const vp_plan* p = s->plan;
    hipStream_t ss = s->stream;
    const KPDesc& d = s->tab.d;
    if (params_out)
        e = hipMemcpyAsync(params_out, d.params, (size_t)d.n_params * sizeof(float2), hipMemcpyDeviceToHost, ss);
    if (e == hipSuccess && n_frames > 0 && (proj_out || water_out || fat_out)) {
        KPTables ft;
        build_tables(p, &s->model, frame_times, n_frames, &ft);
        DevArena ar;
        e = kp_device(&ft, &ar, false, ss);
        const size_t nn = (size_t)p->n * p->n, nf = (size_t)n_frames;
        float2 *vol = nullptr, *pr = nullptr, *wa = nullptr, *fa = nullptr;
        if (e == hipSuccess) e = ar.alloc(&vol, nf * p->S * nn);
        if (e == hipSuccess) e = ar.alloc(&pr, nf * nn);
        if (e == hipSuccess) e = ar.alloc(&wa, nf * nn);
        if (e == hipSuccess) e = ar.alloc(&fa, nf * nn);
        ft.d.params = d.params;
        ft.d.vol = vol;
        const int split = s->opts.split_bin < 0 ? p->S / 2 : s->opts.split_bin;
        if (e == hipSuccess) e = kp_launch_factors(ft.d, ss);
        if (e == hipSuccess) e = kp_launch_decode(ft.d, ss);
        if (e == hipSuccess) e = kp_launch_render(ft.d, split, pr, wa, fa, ss);
        if (e == hipSuccess && proj_out) e = hipMemcpyAsync(proj_out, pr, nf * nn * sizeof(float2), hipMemcpyDeviceToHost, ss);
        if (e == hipSuccess && water_out) e = hipMemcpyAsync(water_out, wa, nf * nn * sizeof(float2), hipMemcpyDeviceToHost, ss);
        if (e == hipSuccess && fat_out) e = hipMemcpyAsync(fat_out, fa, nf * nn * sizeof(float2), hipMemcpyDeviceToHost, ss);
        const hipError_t e2 = hipStreamSynchronize(ss);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && objective) {
        // data term and regularisers at the current parameters (no update)
        if (e == hipSuccess) e = kp_launch_factors(d, ss);
        if (e == hipSuccess) e = kp_launch_decode(d, ss);
        if (e == hipSuccess) e = dense_forward(s->ds, ss);
        if (e == hipSuccess) e = kp_launch_reg_value(d, ss);
        const size_t nl = loss_slots(s->ds.q);
        std::vector<float> hl(nl);
        std::vector<double> hr((size_t)kp_reg_blocks(d));
        if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), s->loss_part, nl * sizeof(float), hipMemcpyDeviceToHost, ss);
        if (e == hipSuccess) e = hipMemcpyAsync(hr.data(), d.rpart, hr.size() * sizeof(double), hipMemcpyDeviceToHost, ss);
        const hipError_t e2 = hipStreamSynchronize(ss);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) {
            *objective = host_objective(hl, hr, nullptr);
            if (!std::isfinite(*objective)) return fail(VP_ERR_NONFINITE, "K-Planes objective is not finite");
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
    return hip_status(e, "vp_kplanes_session_read");
}

extern "C" vp_status vp_kplanes_session_stage_times(vp_kplanes_session* s, int32_t n_steps, double* stage_ms) {
    clear_error();
    if (!s || !stage_ms || n_steps < 1) return fail(VP_ERR_ARG, "vp_kplanes_session_stage_times: bad argument");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    std::vector<hipEvent_t> ev((size_t)n_steps * (kKpStages + 1), nullptr);
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) e = kp_step(s, &ev[(size_t)k * (kKpStages + 1)]);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    for (int i = 0; i < kKpStages; ++i) stage_ms[i] = 0.0;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k)
        for (int i = 0; i < kKpStages && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[(size_t)k * (kKpStages + 1) + i], ev[(size_t)k * (kKpStages + 1) + i + 1]);
            stage_ms[i] += ms / n_steps;
        }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_status(e, "vp_kplanes_session_stage_times");
    s->steps_done += n_steps;
    return VP_OK;
}

namespace {
bool params_finite(const vp_c64* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i].re) || !std::isfinite(a[i].im)) return false;
    return true;
}
}  // namespace

extern "C" vp_status vp_kplanes_session_get_state(vp_kplanes_session* s, vp_c64* params, vp_c64* m, vp_c64* v,
                                                  int64_t* step) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_kplanes_session_get_state: NULL session");
    hipError_t e = hipSetDevice(s->device);
    const KPDesc& d = s->tab.d;
    const size_t pb = (size_t)d.n_params * sizeof(float2);
    if (e == hipSuccess && params) e = hipMemcpyAsync(params, d.params, pb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && m) e = hipMemcpyAsync(m, d.m, pb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && v) e = hipMemcpyAsync(v, d.v, pb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess && step) *step = s->steps_done;
    return hip_status(e, "vp_kplanes_session_get_state");
}

extern "C" vp_status vp_kplanes_session_set_state(vp_kplanes_session* s, const vp_c64* params, const vp_c64* m,
                                                  const vp_c64* v, int64_t step) {
    clear_error();
    if (!s || !params || step < 0 || step > 0x7ffffffe)
        return fail(VP_ERR_ARG, "vp_kplanes_session_set_state: bad argument");
    const KPDesc& d = s->tab.d;
    if (!params_finite(params, (size_t)d.n_params))
        return fail(VP_ERR_NONFINITE, "vp_kplanes_session_set_state: non-finite parameters");
    hipError_t e = hipSetDevice(s->device);
    const size_t pb = (size_t)d.n_params * sizeof(float2);
    const int st32 = (int)step;
    if (e == hipSuccess) e = hipMemcpyAsync((void*)d.params, params, pb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = m ? hipMemcpyAsync(d.m, m, pb, hipMemcpyHostToDevice, s->stream) : hipMemsetAsync(d.m, 0, pb, s->stream);
    if (e == hipSuccess) e = v ? hipMemcpyAsync(d.v, v, pb, hipMemcpyHostToDevice, s->stream) : hipMemsetAsync(d.v, 0, pb, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->step_dev, &st32, sizeof st32, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) s->steps_done = step;
    return hip_status(e, "vp_kplanes_session_set_state");
}

extern "C" vp_status vp_kplanes_session_destroy(vp_kplanes_session* s) {
    if (s) {
        (void)hipSetDevice(s->device);
        delete s;
    }
    return VP_OK;
}

extern "C" vp_status vp_kplanes_reconstruct(const vp_plan* p, const vp_kplanes* m, const vp_options* o,
                                            const vp_c64* kspace, const vp_c64* init, vp_c64* params_out,
                                            int32_t n_frames, const double* frame_times, vp_c64* proj_out,
                                            vp_c64* water_out, vp_c64* fat_out, double* final_loss) {
    vp_kplanes_session* s = nullptr;
    vp_status st = vp_kplanes_session_create(p, m, o, kspace, init, &s);
    if (st != VP_OK) return st;
    st = vp_kplanes_session_step(s, o->n_steps, 1);
    if (st == VP_OK)
        st = vp_kplanes_session_read(s, params_out, n_frames, frame_times, proj_out, water_out, fat_out, final_loss);
    (void)vp_kplanes_session_destroy(s);
    return st;
}
