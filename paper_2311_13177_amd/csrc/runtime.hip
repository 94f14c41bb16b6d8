// Host runtime of libvp: per-device plan tables, operator calls, resident sessions
// (eager or HIP-graph stepping), whole reconstructions and batched reconstructions.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "plan.h"
#include "runtime.h"
#include "nu.h"

namespace vp {

// ------------------------------------------------------------------ device tables

DeviceLayout::~DeviceLayout() {
    void* ptrs[] = {groups, t_proj, t_gath, t_upd};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
}

DeviceTables::~DeviceTables() {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (device >= 0) (void)hipSetDevice(device);
    layouts.clear();
    void* ptrs[] = {mask, shear, blade, knot_ptr, knot_ent, knot_tap, knots, tw, t_rows, t_cols, t_vox, t_render,
                    nu_lines, nu_cs, nu_ph, nu_dea, nu_kb, nu_rows};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (prev >= 0) (void)hipSetDevice(prev);
}

vp_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return VP_OK;
    if (e == hipErrorOutOfMemory) return fail(VP_ERR_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(VP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src) {
    *dst = nullptr;
    const size_t bytes = std::max<size_t>(sizeof(T), src.size() * sizeof(T));
    hipError_t e = hipMalloc((void**)dst, bytes);
    if (e != hipSuccess) return e;
    if (src.empty()) return hipMemset(*dst, 0, bytes);
    return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

vp_status plan_tables(const vp_plan* p, DeviceTables** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->dev.find(dev);
    if (it != p->dev.end()) {
        *out = it->second.get();
        return VP_OK;
    }
    std::unique_ptr<DeviceTables> t(new (std::nothrow) DeviceTables());
    if (!t) return fail(VP_ERR_NOMEM, "plan tables: out of host memory");
    t->device = dev;
#define UP(field, vec)                                         \
    do {                                                       \
        e = upload(&t->field, vec);                            \
        if (e != hipSuccess) return hip_status(e, "plan tables"); \
    } while (0)
    UP(mask, p->mask);
    UP(shear, p->shear);
    UP(blade, p->blade);
    UP(knot_ptr, p->knot_ptr);
    UP(knot_ent, p->knot_ent);
    UP(knot_tap, p->knot_tap);
    UP(knots, p->knots);
    UP(tw, p->tw);
    UP(t_rows, p->t_rows);
    UP(t_cols, p->t_cols);
    UP(t_vox, p->t_vox);
    UP(t_render, p->t_render);
#undef UP
    *out = t.get();
    p->dev.emplace(dev, std::move(t));
    return VP_OK;
}

vp_status device_layout(const vp_plan* p, DeviceTables* t, const Layout* L, const DeviceLayout** out) {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = t->layouts.find(L->tiles.key());
    if (it != t->layouts.end()) {
        *out = it->second.get();
        return VP_OK;
    }
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (prev != t->device && (e = hipSetDevice(t->device)) != hipSuccess) return hip_status(e, "hipSetDevice");
    std::unique_ptr<DeviceLayout> d(new (std::nothrow) DeviceLayout());
    if (!d) return fail(VP_ERR_NOMEM, "layout tables: out of host memory");
    e = upload(&d->groups, L->groups);
    if (e == hipSuccess) e = upload(&d->t_proj, L->t_proj);
    if (e == hipSuccess) e = upload(&d->t_gath, L->t_gath);
    if (e == hipSuccess) e = upload(&d->t_upd, L->t_upd);
    if (prev != t->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return hip_status(e, "layout tables");
    *out = d.get();
    t->layouts.emplace(L->tiles.key(), std::move(d));
    return VP_OK;
}

void fill_desc(const vp_plan* p, const DeviceTables* t, const Layout* L, const DeviceLayout* dl, SliceDesc* d) {
    std::memset(d, 0, sizeof *d);
    d->n = p->n;
    d->S = p->S;
    d->T = p->T;
    d->B = p->B;
    d->nparts = p->nparts;
    d->nstage = p->nstage;
    for (int i = 0; i < kMaxStages; ++i) d->radix[i] = p->radix[i];
    d->radix_code = 0;
    for (int i = 0; i < p->nstage; ++i) d->radix_code |= p->radix[i] << (3 * i);
    d->n_col_items = p->n_col_items;
    d->tw = t->tw;
    d->mask = t->mask;
    d->shear = t->shear;
    d->blade = t->blade;
    d->knot_ptr = t->knot_ptr;
    d->knot_ent = t->knot_ent;
    d->knot_tap = t->knot_tap;
    d->groups = dl->groups;
    d->knots = t->knots;
    d->step_limit = 0x7fffffff;
    d->schedule = VP_SCHED_ALL_BLADES;
    d->sched_seed = 0;
    d->data_w = 1.0f;
    d->optimizer = VP_OPT_ADAM;
}

static void set_hyper(SliceDesc* d, const vp_options* o) {
    d->optimizer = o->optimizer;
    d->schedule = o->schedule;
    d->sched_seed = o->seed;
    d->data_w = o->data_weight;
    d->lr = o->lr;
    d->beta1 = o->beta1;
    d->beta2 = o->beta2;
    d->ln_beta1 = (float)std::log((double)o->beta1);
    d->ln_beta2 = (float)std::log((double)o->beta2);
    d->adam_eps = o->adam_eps;
    d->tv_w = o->tv_weight;
    d->l1_w = o->l1_weight;
    d->tv_eps = o->tv_eps;
}

vp_status check_options(const vp_plan* p, const vp_options* o) {
    if (!o) return fail(VP_ERR_ARG, "NULL options");
    const float fs[] = {o->tv_weight, o->l1_weight, o->tv_eps, o->lr, o->beta1, o->beta2, o->adam_eps, o->data_weight};
    for (float f : fs)
        if (!std::isfinite(f)) return fail(VP_ERR_ARG, "options: non-finite value");
    if (o->tv_weight < 0 || o->l1_weight < 0 || o->tv_eps <= 0)
        return fail(VP_ERR_ARG, "options: weights must be >= 0 and tv_eps > 0");
    if (o->n_steps < 0) return fail(VP_ERR_ARG, "options: n_steps < 0");
    if (o->optimizer != VP_OPT_ADAM && o->optimizer != VP_OPT_GD) return fail(VP_ERR_ARG, "options: optimizer");
    if (o->schedule != VP_SCHED_ALL_BLADES && o->schedule != VP_SCHED_CYCLIC && o->schedule != VP_SCHED_RANDOM)
        return fail(VP_ERR_ARG, "options: schedule");
    if (!(o->data_weight > 0)) return fail(VP_ERR_ARG, "options: data_weight must be > 0");
    if (o->optimizer == VP_OPT_ADAM && (o->beta1 < 0 || o->beta1 >= 1 || o->beta2 < 0 || o->beta2 >= 1))
        return fail(VP_ERR_ARG, "options: betas must lie in [0, 1)");
    if (o->split_bin > p->S) return fail(VP_ERR_ARG, "options: split_bin above n_spec");
    const vp_tiles& t = o->tiles;
    const bool none = !t.proj_rows && !t.proj_parts && !t.gath_rows && !t.gath_bins && !t.upd_bins && !t.gath_waves &&
                      !t.proj_waves && !t.gath_resident;
    if (!none && (!proj_tiles_ok(t.proj_rows, t.proj_parts) || !gath_tiles_ok(t.gath_rows, t.gath_bins, t.gath_resident == 1) ||
                  !upd_tiles_ok(t.upd_bins) || (t.gath_waves != 0 && !item_waves_ok(t.gath_waves)) ||
                  (t.proj_waves != 0 && !item_waves_ok(t.proj_waves)) || (t.gath_resident != 0 && t.gath_resident != 1) ||
                  (t.gath_resident && t.upd_bins)))
        return fail(VP_ERR_UNSUPPORTED, "options: tile shape (%d, %d, %d, %d, %d, %d, %d, %d) is not compiled",
                    t.proj_rows, t.proj_parts, t.gath_rows, t.gath_bins, t.upd_bins, t.gath_waves, t.proj_waves,
                    t.gath_resident);
    return VP_OK;
}

// ------------------------------------------------------------------ launch sequences

void launch_step(const KArgs& base, const StageLists& L, hipStream_t s, hipError_t* err, hipEvent_t* ev) {
    // the projection takes the step counters' snapshot and the step's last kernel advances
    // them from it: both launches must have work items (every plan has, by construction)
    if (L.n_proj <= 0 || (L.tiles.upd_sc == 0 ? L.n_gath <= 0 : L.n_upd <= 0)) {
        *err = hipErrorInvalidValue;
        return;
    }
    KArgs a = base;
    a.epi = L.epi;
    a.stream = L.stream;
    hipError_t e;
#define MARK(i)                                                                         \
    do {                                                                                \
        if (ev && (e = hipEventRecord(ev[i], s)) != hipSuccess) { *err = e; return; }  \
    } while (0)
    MARK(0);
    // the projection snapshots the step counters, the last kernel reads the snapshot and
    // advances them (step_snapshot, step_advance)
    a.nslices = L.n_slices;
    a.snap = 1;
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, s)) != hipSuccess) { *err = e; return; }
    a.snap = 0;
    MARK(1);
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, -1, L.fft_n, L.lds_rows, s)) != hipSuccess) { *err = e; return; }
    MARK(2);
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_STEP;
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, s)) != hipSuccess) { *err = e; return; }
    MARK(3);
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, 1, L.fft_n, L.lds_rows, s)) != hipSuccess) { *err = e; return; }
    MARK(4);
    a.tasks = L.gath; a.ntasks = L.n_gath;
    a.snap = 1;
    if (L.tiles.upd_sc == 0) {
        a.advance = 1;
        e = launch_gather_lists(a, GATHER_STEP, L, s);
    } else {
        a.accumulate = 0;
        e = launch_gather_lists(a, GATHER_STORE, L, s);
        a.tasks = L.upd; a.ntasks = L.n_upd; a.advance = 1;
        if (e == hipSuccess) e = launch_update(a, L.tiles.upd_sc, s);
    }
    if (e != hipSuccess) {
        *err = e;
        return;
    }
    MARK(5);
#undef MARK
    *err = hipSuccess;
}

StageLists plan_lists(const vp_plan* p, const DeviceTables* t, const Layout* lay, const DeviceLayout* dl) {
    StageLists L;
    L.proj = dl->t_proj; L.n_proj = (int)lay->t_proj.size();
    L.rows = t->t_rows; L.n_rows = (int)p->t_rows.size();
    L.cols = t->t_cols; L.n_cols = (int)p->t_cols.size();
    L.gath = dl->t_gath; L.n_gath = (int)lay->t_gath.size();
    L.upd = dl->t_upd; L.n_upd = (int)lay->t_upd.size();
    L.vox = t->t_vox; L.n_vox = (int)p->t_vox.size();
    L.render = t->t_render; L.n_render = (int)p->t_render.size();
    L.tiles = lay->tiles;
    L.fft_n = p->n;
    L.re_proj = lay->re_proj; L.lds_rows = p->lds_rows; L.lds_cols = p->lds_cols; L.re_gath = lay->re_gath;
    L.lds_res = lay->lds_res;
    return L;
}

}  // namespace vp

using namespace vp;

// ------------------------------------------------------------------ plans

extern "C" vp_status vp_plan_destroy(vp_plan* p) {
    delete p;
    return VP_OK;
}

// ------------------------------------------------------------------ operators

namespace {

// Operator calls use the tuned tile shape recorded for the plan's sizes on the current
// device, else the plan's heuristic shape.
struct OpScope {
    const vp_plan* p;
    DeviceTables* t = nullptr;
    const Layout* lay = nullptr;
    const DeviceLayout* dl = nullptr;
    hipStream_t s;
    float2* work = nullptr;
    explicit OpScope(const vp_plan* plan, void* stream) : p(plan), s((hipStream_t)stream) {}
    vp_status begin(bool need_work) {
        vp_status st = plan_tables(p, &t);
        if (st != VP_OK) return st;
        Tiles tl = p->base_tiles;
        (void)tuned_tiles(p, t->device, VP_OPT_ADAM, &tl);
        st = plan_layout(p, tl, &lay);
        if (st != VP_OK) st = plan_layout(p, p->base_tiles, &lay);
        if (st == VP_OK) st = device_layout(p, t, lay, &dl);
        if (st != VP_OK) return st;
        if (need_work) {
            const size_t bytes = (size_t)p->nparts * p->blade_px() * sizeof(float2);
            hipError_t e = hipMallocAsync((void**)&work, bytes, s);
            if (e != hipSuccess) return hip_status(e, "workspace");
        }
        return VP_OK;
    }
    ~OpScope() {
        if (work) (void)hipFreeAsync(work, s);
    }
};

}  // namespace

extern "C" vp_status vp_forward(const vp_plan* p, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out,
                                void* stream) {
    clear_error();
    if (!p || !d_vol || !d_out) return fail(VP_ERR_ARG, "vp_forward: NULL argument");
    OpScope sc(p, stream);
    vp_status st = sc.begin(true);
    if (st != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.vol[0] = (float2*)d_vol;
    a.one.y = (const float2*)d_y;
    a.one.work = sc.work;
    const StageLists L = plan_lists(p, sc.t, sc.lay, sc.dl);
    hipError_t e;
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, sc.s)) != hipSuccess)
        return hip_status(e, "vp_forward project");
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, -1, L.fft_n, L.lds_rows, sc.s)) != hipSuccess) return hip_status(e, "vp_forward rows");
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_FORWARD; a.out0 = (float2*)d_out;
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, sc.s)) != hipSuccess) return hip_status(e, "vp_forward cols");
    return VP_OK;
}

extern "C" vp_status vp_adjoint(const vp_plan* p, const vp_c64* d_kres, vp_c64* d_grad, int32_t accumulate,
                                void* stream) {
    clear_error();
    if (!p || !d_kres || !d_grad) return fail(VP_ERR_ARG, "vp_adjoint: NULL argument");
    OpScope sc(p, stream);
    vp_status st = sc.begin(true);
    if (st != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.work = sc.work;
    a.one.grad = (float2*)d_grad;
    a.accumulate = accumulate != 0;
    const StageLists L = plan_lists(p, sc.t, sc.lay, sc.dl);
    hipError_t e;
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_ADJOINT; a.in0 = (const float2*)d_kres;
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, sc.s)) != hipSuccess) return hip_status(e, "vp_adjoint cols");
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, 1, L.fft_n, L.lds_rows, sc.s)) != hipSuccess) return hip_status(e, "vp_adjoint rows");
    a.tasks = L.gath; a.ntasks = L.n_gath;
    if ((e = launch_gather_lists(a, GATHER_STORE, L, sc.s)) != hipSuccess)
        return hip_status(e, "vp_adjoint gather");
    return VP_OK;
}

// ------------------------------------------------------------------ forward without allocation
//
// vp_forward_noalloc runs vp_forward's kernels with the blade work images in a
// file-scope device array instead of stream-ordered memory. Each device holds its own
// copy of the array at its own address: host code takes that address from
// hipGetSymbolAddress (once per device, on the first call there) and passes it to the
// kernels; the array's name is never used as a device address on the host.

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
__device__ __align__(256) float2 scratch[kScratchBytes / sizeof(float2)];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
float2* g_scratch_ptr[kScratchDevices] = {};

// This device's copy of the scratch array (the current device is `dev`).
vp_status scratch_address(int dev, float2** out) {
    if (dev < 0 || dev >= kScratchDevices) return fail(VP_ERR_DEVICE, "vp_forward_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
        g_scratch_ptr[dev] = (float2*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return VP_OK;
}

// The device tables and the layout an operator call would use on `dev`, when both exist
// already: nothing is built, uploaded or allocated here.
vp_status existing_tables(const vp_plan* p, int dev, const DeviceTables** t, const Layout** lay,
                          const DeviceLayout** dl) {
    Tiles want = p->base_tiles;
    (void)tuned_tiles(p, dev, VP_OPT_ADAM, &want);
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->dev.find(dev);
    if (it == p->dev.end())
        return fail(VP_ERR_STATE, "vp_forward_noalloc: the plan has no tables on device %d yet", dev);
    const DeviceTables* tab = it->second.get();
    for (const Tiles& tl : {want, p->base_tiles}) {
        auto hl = p->layouts.find(tl.key());
        auto dlit = tab->layouts.find(tl.key());
        if (hl != p->layouts.end() && dlit != tab->layouts.end()) {
            *t = tab;
            *lay = hl->second.get();
            *dl = dlit->second.get();
            return VP_OK;
        }
    }
    return fail(VP_ERR_STATE, "vp_forward_noalloc: the plan's launch tables are not on device %d yet", dev);
}

}  // namespace

extern "C" vp_status vp_forward_noalloc(const vp_plan* p, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out,
                                        void* stream) {
    clear_error();
    if (!p || !d_vol || !d_out) return fail(VP_ERR_ARG, "vp_forward_noalloc: NULL argument");
    const size_t bytes = (size_t)p->nparts * p->blade_px() * sizeof(float2);
    if (bytes > kScratchBytes)
        return fail(VP_ERR_UNSUPPORTED, "vp_forward_noalloc: %zu bytes of blade images exceed the %zu-byte scratch",
                    bytes, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    const DeviceTables* t = nullptr;
    const Layout* lay = nullptr;
    const DeviceLayout* dl = nullptr;
    vp_status st = existing_tables(p, dev, &t, &lay, &dl);
    if (st != VP_OK) return st;
    float2* work = nullptr;
    if ((st = scratch_address(dev, &work)) != VP_OK) return st;
    const hipStream_t s = (hipStream_t)stream;
    KArgs a{};
    fill_desc(p, t, lay, dl, &a.one);
    a.one.vol[0] = (float2*)d_vol;
    a.one.y = (const float2*)d_y;
    a.one.work = work;
    const StageLists L = plan_lists(p, t, lay, dl);
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, s)) != hipSuccess)
        return hip_status(e, "vp_forward_noalloc project");
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, -1, L.fft_n, L.lds_rows, s)) != hipSuccess) return hip_status(e, "vp_forward_noalloc rows");
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_FORWARD; a.out0 = (float2*)d_out;
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, s)) != hipSuccess) return hip_status(e, "vp_forward_noalloc cols");
    return VP_OK;
}

// Section 6 baselines: the coverage-weighted average (scaled by 1/n) into d_out, then the
// inverse column and row DFTs in place, over the frames' prefix of the work lists.
extern "C" vp_status vp_baseline(const vp_plan* p, const vp_c64* d_kspace, int32_t window, int32_t first_frame,
                                 int32_t n_frames, vp_c64* d_out, void* stream) {
    clear_error();
    if (!p) return fail(VP_ERR_ARG, "vp_baseline: NULL plan");
    if (first_frame < 0 || n_frames < 0 || (int64_t)first_frame + n_frames > p->B)
        return fail(VP_ERR_ARG, "vp_baseline: frames outside [0, B)");
    if (n_frames == 0) return VP_OK;
    if (!d_kspace || !d_out) return fail(VP_ERR_ARG, "vp_baseline: NULL argument");
    const size_t nn = (size_t)p->n * p->n;
    const uintptr_t k0 = (uintptr_t)d_kspace, k1 = k0 + (size_t)p->B * nn * sizeof(vp_c64);
    const uintptr_t o0 = (uintptr_t)d_out, o1 = o0 + (size_t)n_frames * nn * sizeof(vp_c64);
    if (o0 < k1 && k0 < o1) return fail(VP_ERR_ARG, "vp_baseline: d_out overlaps d_kspace");
    OpScope sc(p, stream);
    vp_status st = sc.begin(false);
    if (st != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    const StageLists L = plan_lists(p, sc.t, sc.lay, sc.dl);
    hipError_t e = launch_baseline_avg(sc.t->mask, (const float2*)d_kspace, (float2*)d_out, p->n, window,
                                       first_frame, n_frames, sc.s);
    if (e != hipSuccess) return hip_status(e, "vp_baseline average");
    a.mode = COL_INVERSE;
    a.in0 = (const float2*)d_out;
    a.out0 = (float2*)d_out;
    a.tasks = L.cols; a.ntasks = n_frames * (L.n_cols / p->B);
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, sc.s)) != hipSuccess) return hip_status(e, "vp_baseline cols");
    a.tasks = L.rows; a.ntasks = n_frames * (L.n_rows / p->B);
    if ((e = launch_rows(a, 1, L.fft_n, L.lds_rows, sc.s)) != hipSuccess) return hip_status(e, "vp_baseline rows");
    return VP_OK;
}

extern "C" vp_status vp_psnr(const vp_c64* d_image, const vp_c64* d_truth, int64_t n_px, int32_t n_images,
                             double* d_terms, void* stream) {
    clear_error();
    if (n_px < 1 || n_images < 0) return fail(VP_ERR_ARG, "vp_psnr: n_px < 1 or n_images < 0");
    if (n_images == 0) return VP_OK;
    if (!d_image || !d_truth || !d_terms) return fail(VP_ERR_ARG, "vp_psnr: NULL argument");
    const hipError_t e = launch_psnr((const float2*)d_image, (const float2*)d_truth, (long long)n_px, n_images,
                                     d_terms, (hipStream_t)stream);
    return e == hipSuccess ? VP_OK : hip_status(e, "vp_psnr");
}

// ------------------------------------------------------------------ blade-aligned sampling

namespace vp {

vp_status nu_tables(const vp_plan* p, const NuHost* h, DeviceTables* t) {
    std::lock_guard<std::mutex> lk(p->mu);
    if (t->nu_kb) return VP_OK;
    hipError_t e = upload(&t->nu_lines, h->lines);
    if (e == hipSuccess) e = upload(&t->nu_cs, h->cs);
    if (e == hipSuccess) e = upload(&t->nu_ph, h->ph);
    if (e == hipSuccess) e = upload(&t->nu_dea, h->dea);
    if (e == hipSuccess) e = upload(&t->nu_kb, h->kb);
    if (e == hipSuccess) e = upload(&t->nu_rows, h->rows);
    return hip_status(e, "blade sampling tables");
}

}  // namespace vp

namespace {

// The oversampled grid's plan and its DFT passes, plus the gridding arguments.
struct NuScope {
    const vp_plan* q = nullptr;
    DeviceTables* tq = nullptr;
    const Layout* lq = nullptr;
    const DeviceLayout* dq = nullptr;
    const NuHost* h = nullptr;
    float2* grid = nullptr;
    const Task* t_img_rows = nullptr;  // row-pass tasks over the image's rows only
    // a fit's one-blade schedule: the DFT passes skip inactive blades as the other passes do
    int sched = VP_SCHED_ALL_BLADES;
    unsigned sseed = 0;
    int* stepp = nullptr;
    hipStream_t s;
    bool persistent = false;  // grids from hipMalloc (a fit), else stream-ordered (an operator call)
    NuArgs d{};
    explicit NuScope(hipStream_t stream, bool keep = false) : s(stream), persistent(keep) {}
    vp_status begin(const vp_plan* p, DeviceTables* t) {
        vp_status st = plan_nu(p, &h, &q);
        if (st == VP_OK) st = nu_tables(p, h, t);
        if (st == VP_OK) st = plan_tables(q, &tq);
        if (st == VP_OK) st = plan_layout(q, q->base_tiles, &lq);
        if (st == VP_OK) st = device_layout(q, tq, lq, &dq);
        if (st != VP_OK) return st;
        // the grids, then the premultiplied samples the spread reads
        const size_t ngrid = (size_t)p->B * q->n * q->n, nsamp = (size_t)p->B * h->lmax * p->n;
        const size_t bytes = (ngrid + nsamp) * sizeof(float2);
        hipError_t e = persistent ? hipMalloc((void**)&grid, bytes) : hipMallocAsync((void**)&grid, bytes, s);
        if (e != hipSuccess) return hip_status(e, "oversampled grids");
        d.n = p->n; d.M = q->n; d.B = p->B; d.lmax = h->lmax; d.nparts = p->nparts; d.kmax = h->kmax;
        d.dw = 1.0f;
        d.lines = t->nu_lines; d.cs = t->nu_cs; d.dea = t->nu_dea; d.kb = t->nu_kb;  d.ph = t->nu_ph;
        d.blade = t->blade;
        d.grid = grid;
        d.pre = grid + ngrid;
        t_img_rows = t->nu_rows;
        return VP_OK;
    }
    // The unscaled 2D DFT of the grids, in four passes: the forward row pass builds the
    // image rows of the grids from the blade images (centred, deapodised; the other rows
    // stay unread), the forward column pass completes the DFT in place; the inverse column
    // pass writes only the image rows, and the inverse row pass writes their centres,
    // deapodised, into the blade images (part 0).
    hipError_t pass(int which) {
        KArgs a{};
        fill_desc(q, tq, lq, dq, &a.one);
        const StageLists L = plan_lists(q, tq, lq, dq);
        a.in0 = grid;
        a.out0 = grid;
        a.live_n = d.n;
        a.nue.img_in = d.work;
        a.nue.img_out = d.img_out;
        a.nue.blade = d.blade;
        a.nue.dea = d.dea;
        a.nue.parts = d.nparts;
        a.one.schedule = sched;
        a.one.sched_seed = sseed;
        a.one.step = stepp;
        a.one.step_limit = 0x7fffffff;
        a.mode = which < 2 ? COL_RAW_FWD : COL_INVERSE;
        if (which == 1 || which == 2) {
            a.tasks = L.cols; a.ntasks = L.n_cols;
            return launch_cols(a, L.fft_n, (size_t)fft_cols_raw_lds(q->n), s);
        }
        a.tasks = t_img_rows; a.ntasks = (int)h->rows.size();
        return launch_rows(a, which == 0 ? -1 : 1, L.fft_n, L.lds_rows, s);
    }
    enum { ROWS_FWD = 0, COLS_FWD = 1, COLS_INV = 2, ROWS_INV = 3 };
    ~NuScope() {
        if (!grid) return;
        if (persistent) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(grid);
        } else {
            (void)hipFreeAsync(grid, s);
        }
    }
};

}  // namespace

extern "C" vp_status vp_nu_forward(const vp_plan* p, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out,
                                   void* stream) {
    clear_error();
    if (!p || !d_vol || !d_out) return fail(VP_ERR_ARG, "vp_nu_forward: NULL argument");
    OpScope sc(p, stream);
    vp_status st = sc.begin(true);
    if (st != VP_OK) return st;
    NuScope nu(sc.s);
    if ((st = nu.begin(p, sc.t)) != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.vol[0] = (float2*)d_vol;
    a.one.work = sc.work;
    const StageLists L = plan_lists(p, sc.t, sc.lay, sc.dl);
    hipError_t e;
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, sc.s)) != hipSuccess)
        return hip_status(e, "vp_nu_forward project");
    nu.d.work = sc.work;
    nu.d.y = (const float2*)d_y;
    nu.d.out = (float2*)d_out;
    nu.d.pre = nullptr;
    if ((e = nu.pass(NuScope::ROWS_FWD)) != hipSuccess || (e = nu.pass(NuScope::COLS_FWD)) != hipSuccess)
        return hip_status(e, "vp_nu_forward DFT");
    if ((e = nu_launch_interp(nu.d, sc.s)) != hipSuccess) return hip_status(e, "vp_nu_forward interpolation");
    return VP_OK;
}

extern "C" vp_status vp_nu_adjoint(const vp_plan* p, const vp_c64* d_samples, vp_c64* d_grad, int32_t accumulate,
                                   void* stream) {
    clear_error();
    if (!p || !d_samples || !d_grad) return fail(VP_ERR_ARG, "vp_nu_adjoint: NULL argument");
    OpScope sc(p, stream);
    vp_status st = sc.begin(true);
    if (st != VP_OK) return st;
    NuScope nu(sc.s);
    if ((st = nu.begin(p, sc.t)) != VP_OK) return st;
    hipError_t e;
    nu.d.s_in = (const float2*)d_samples;
    nu.d.img_out = sc.work;
    if ((e = nu_launch_prep(nu.d, sc.s)) != hipSuccess) return hip_status(e, "vp_nu_adjoint prep");
    if ((e = nu_launch_spread(nu.d, sc.s)) != hipSuccess) return hip_status(e, "vp_nu_adjoint spread");
    if ((e = nu.pass(NuScope::COLS_INV)) != hipSuccess || (e = nu.pass(NuScope::ROWS_INV)) != hipSuccess)
        return hip_status(e, "vp_nu_adjoint DFT");
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.work = sc.work;
    a.one.grad = (float2*)d_grad;
    a.accumulate = accumulate != 0;
    const StageLists L = plan_lists(p, sc.t, sc.lay, sc.dl);
    a.tasks = L.gath; a.ntasks = L.n_gath;
    if ((e = launch_gather_lists(a, GATHER_STORE, L, sc.s)) != hipSuccess)
        return hip_status(e, "vp_nu_adjoint gather");
    return VP_OK;
}

// A fit on blade-aligned samples: the session's projection, gather and fused update with
// the gridding passes in place of the Cartesian DFT passes (all blades every step).
// ------------------------------------------------------------------ fits on blade-aligned samples

namespace {
// project, forward rows, forward columns, interp, spread, inverse columns, inverse rows,
// gather+update
constexpr int kNuStages = 8;
}

// A Cartesian session (volume, optimiser state, projection and gather lists, step counter)
// whose data term runs through the gridding passes: per step project, the forward DFT of
// the grids (its row pass builds the grid rows from the blade images), interpolate minus
// the samples (with loss partials), spread, the inverse DFT (its row pass writes the blade
// images), then the fused gather with the regulariser gradient and update, and the counter.
struct vp_nu_session {
    std::unique_ptr<vp_session> s;
    NuScope nu;
    float2* res = nullptr;  // residual samples [B][Lmax][n]
    float2* ys = nullptr;   // measured samples [B][Lmax][n]
    float* loss = nullptr;  // per-block sums of |residual|^2 of the last forward pass
    int nblk = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    explicit vp_nu_session(vp_session* raw) : s(raw), nu(raw->stream, true) {}
    ~vp_nu_session() {
        (void)hipSetDevice(s->device);
        (void)hipStreamSynchronize(s->stream);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        void* bufs[] = {res, ys, loss};
        for (void* q : bufs)
            if (q) (void)hipFree(q);
    }

    // the schedule the gridding passes follow: the fit's, or all blades (the objective)
    void schedule(bool all) {
        nu.sched = all ? (int)VP_SCHED_ALL_BLADES : s->opts.schedule;
        nu.sseed = s->opts.seed;
        nu.stepp = s->desc.step;
        nu.d.sched = nu.sched;
        nu.d.sseed = nu.sseed;
        nu.d.stepp = nu.stepp;
    }

    // projection to residual samples (and their loss partials) at the current volume, over
    // the fit's blades or all of them; ev (may be null) gets events 0..3 before the first
    // four stages
    hipError_t forward(hipEvent_t* ev, bool all = false) {
        const StageLists& L = s->lists;
        const hipStream_t str = s->stream;
        KArgs a{};
        a.one = s->desc;
        if (all) {
            a.one.schedule = VP_SCHED_ALL_BLADES;
            a.one.step_limit = 0x7fffffff;
        }
        a.tasks = L.proj; a.ntasks = L.n_proj;
        a.snap = 1;  // snapshot of the step counter for the step's last kernel
        a.nslices = 1;
        hipError_t r = ev ? hipEventRecord(ev[0], str) : hipSuccess;
        if (r == hipSuccess) r = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, str);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[1], str);
        if (r == hipSuccess) r = nu.pass(NuScope::ROWS_FWD);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[2], str);
        if (r == hipSuccess) r = nu.pass(NuScope::COLS_FWD);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[3], str);
        if (r == hipSuccess) r = nu_launch_interp(nu.d, str);
        return r;
    }

    // one optimiser step; ev (may be null) gets kNuStages + 1 events around the stages
    hipError_t step(hipEvent_t* ev) {
        const StageLists& L = s->lists;
        const hipStream_t str = s->stream;
        hipError_t r = forward(ev);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[4], str);
        if (r == hipSuccess) r = nu_launch_spread(nu.d, str);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[5], str);
        if (r == hipSuccess) r = nu.pass(NuScope::COLS_INV);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[6], str);
        if (r == hipSuccess) r = nu.pass(NuScope::ROWS_INV);
        if (r == hipSuccess && ev) r = hipEventRecord(ev[7], str);
        KArgs a{};
        a.one = s->desc;
        a.epi = L.epi;
        a.stream = L.stream;
        a.tasks = L.gath; a.ntasks = L.n_gath;
        a.snap = 1;  // the last kernel reads the snapshot and advances the counter
        a.nslices = 1;
        if (r == hipSuccess) {
            if (L.tiles.upd_sc == 0) {
                a.advance = 1;
                r = launch_gather_lists(a, GATHER_STEP, L, str);
            } else {
                r = launch_gather_lists(a, GATHER_STORE, L, str);
                a.tasks = L.upd; a.ntasks = L.n_upd; a.advance = 1;
                if (r == hipSuccess) r = launch_update(a, L.tiles.upd_sc, str);
            }
        }
        if (r == hipSuccess && ev) r = hipEventRecord(ev[kNuStages], str);
        return r;
    }
};

extern "C" vp_status vp_nu_session_create(const vp_plan* p, const vp_options* o, const vp_c64* samples,
                                          const vp_c64* init, vp_nu_session** out) {
    clear_error();
    if (!p || !o || !samples || !out) return fail(VP_ERR_ARG, "vp_nu_session_create: NULL argument");
    *out = nullptr;
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    const NuHost* h = nullptr;
    const vp_plan* q = nullptr;
    if ((st = plan_nu(p, &h, &q)) != VP_OK) return st;
    const size_t ns = (size_t)p->B * h->lmax * p->n;
    for (int b = 0; b < p->B; ++b)
        for (size_t i = (size_t)b * h->lmax * p->n; i < ((size_t)b * h->lmax + p->lines[b]) * p->n; ++i)
            if (!std::isfinite(samples[i].re) || !std::isfinite(samples[i].im))
                return fail(VP_ERR_NONFINITE, "vp_nu_session_create: samples hold NaN or Inf");
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    std::vector<vp_c64> zeros;
    try {
        zeros.assign(p->blade_px(), vp_c64{0.f, 0.f});
    } catch (const std::bad_alloc&) {
        return fail(VP_ERR_NOMEM, "vp_nu_session_create: out of host memory");
    }
    vp_session* raw = nullptr;
    if ((st = session_alloc(p, o, zeros.data(), init, nullptr, &raw)) != VP_OK) return st;
    std::unique_ptr<vp_nu_session> ns_(new (std::nothrow) vp_nu_session(raw));
    if (!ns_) {
        delete raw;
        return fail(VP_ERR_NOMEM, "vp_nu_session_create: out of host memory");
    }
    vp_nu_session* x = ns_.get();
    if ((st = x->nu.begin(p, x->s->tabs)) != VP_OK) return st;
    x->nblk = nu_interp_blocks(x->nu.d);
    e = hipMalloc((void**)&x->res, ns * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&x->ys, ns * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc((void**)&x->loss, x->nblk * sizeof(float));
    if (e == hipSuccess) e = hipMemcpyAsync(x->ys, samples, ns * sizeof(float2), hipMemcpyHostToDevice, x->s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(x->s->stream);
    if (e != hipSuccess) return hip_status(e, "vp_nu_session_create buffers");
    NuArgs& d = x->nu.d;
    d.work = x->s->work;
    d.img_out = x->s->work;
    d.y = x->ys;
    d.out = x->res;
    d.dw = o->data_weight;  // interp writes the spread's input to d.pre
    d.loss = x->loss;
    x->schedule(false);
    *out = ns_.release();
    return VP_OK;
}

extern "C" vp_status vp_nu_session_step(vp_nu_session* x, int32_t n_steps, int32_t use_graph) {
    clear_error();
    if (!x || n_steps < 0) return fail(VP_ERR_ARG, "vp_nu_session_step: bad argument");
    hipError_t e = hipSetDevice(x->s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    const hipStream_t str = x->s->stream;
    if (use_graph && n_steps > 1 && !x->gexec) {
        e = hipStreamBeginCapture(str, hipStreamCaptureModeThreadLocal);
        const hipError_t le = e == hipSuccess ? x->step(nullptr) : e;
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(str, &g);
        if (e == hipSuccess) e = le != hipSuccess ? le : ce;
        x->graph = g;
        if (e == hipSuccess) e = hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) return hip_status(e, "vp_nu_session_step capture");
    }
    for (int i = 0; i < n_steps && e == hipSuccess; ++i)
        e = (use_graph && x->gexec) ? hipGraphLaunch(x->gexec, str) : x->step(nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(str);
    if (e != hipSuccess) return hip_status(e, "vp_nu_session_step");
    x->s->steps_done += n_steps;
    return VP_OK;
}

extern "C" vp_status vp_nu_session_stage_times(vp_nu_session* x, int32_t n_steps, double* stage_ms) {
    clear_error();
    if (!x || !stage_ms || n_steps < 1) return fail(VP_ERR_ARG, "vp_nu_session_stage_times: bad argument");
    hipError_t e = hipSetDevice(x->s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    std::vector<hipEvent_t> ev((size_t)n_steps * (kNuStages + 1), nullptr);
    for (auto& v : ev)
        if (e == hipSuccess) e = hipEventCreate(&v);
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) e = x->step(&ev[(size_t)k * (kNuStages + 1)]);
    if (e == hipSuccess) e = hipStreamSynchronize(x->s->stream);
    for (int i = 0; i < kNuStages; ++i) stage_ms[i] = 0.0;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k)
        for (int i = 0; i < kNuStages && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[(size_t)k * (kNuStages + 1) + i], ev[(size_t)k * (kNuStages + 1) + i + 1]);
            stage_ms[i] += ms / n_steps;
        }
    for (auto& v : ev)
        if (v) (void)hipEventDestroy(v);
    if (e != hipSuccess) return hip_status(e, "vp_nu_session_stage_times");
    x->s->steps_done += n_steps;
    return VP_OK;
}

extern "C" vp_status vp_nu_session_read(vp_nu_session* x, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out,
                                        vp_c64* fat_out, double* objective) {
    clear_error();
    if (!x) return fail(VP_ERR_ARG, "vp_nu_session_read: NULL session");
    hipError_t e = hipSetDevice(x->s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    if (objective) {
        vp_session* s = x->s.get();
        const vp_plan* p = s->plan;
        x->schedule(true);
        e = x->forward(nullptr, true);
        x->schedule(false);
        KArgs a{};
        a.one = s->desc;
        a.tasks = s->lists.vox; a.ntasks = s->lists.n_vox; a.dpart = s->dpart;
        if (e == hipSuccess) e = launch_reg_value(a, s->stream);
        std::vector<float> hl(x->nblk);
        std::vector<double> hd(2 * p->t_vox.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(hl.data(), x->loss, x->nblk * sizeof(float), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(hd.data(), s->dpart, hd.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_status(e, "vp_nu_session_read objective");
        double data = 0.0, tv = 0.0, l1 = 0.0;
        for (float v : hl) data += (double)v;
        for (size_t i = 0; i < p->t_vox.size(); ++i) {
            tv += hd[2 * i];
            l1 += hd[2 * i + 1];
        }
        const vp_options& o = s->opts;
        *objective = 0.5 * (double)o.data_weight * data + (double)o.tv_weight * tv + (double)o.l1_weight * l1;
        if (!std::isfinite(*objective)) return fail(VP_ERR_NONFINITE, "vp_nu_session_read: objective is not finite");
    }
    return session_read(x->s.get(), volume_out, proj_out, water_out, fat_out);
}

extern "C" vp_status vp_nu_session_get_state(vp_nu_session* x, vp_c64* volume, vp_c64* m, vp_c64* v,
                                             int64_t* step) {
    if (!x) {
        clear_error();
        return fail(VP_ERR_ARG, "vp_nu_session_get_state: NULL session");
    }
    return vp_session_get_state(x->s.get(), volume, m, v, step);
}

extern "C" vp_status vp_nu_session_set_state(vp_nu_session* x, const vp_c64* volume, const vp_c64* m,
                                             const vp_c64* v, int64_t step) {
    if (!x) {
        clear_error();
        return fail(VP_ERR_ARG, "vp_nu_session_set_state: NULL session");
    }
    return vp_session_set_state(x->s.get(), volume, m, v, step);
}

extern "C" vp_status vp_nu_session_destroy(vp_nu_session* x) {
    delete x;
    return VP_OK;
}

extern "C" vp_status vp_nu_reconstruct(const vp_plan* p, const vp_options* o, const vp_c64* samples,
                                       const vp_c64* init, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out,
                                       vp_c64* fat_out, double* final_loss) {
    vp_nu_session* x = nullptr;
    vp_status st = vp_nu_session_create(p, o, samples, init, &x);
    if (st != VP_OK) return st;
    st = vp_nu_session_step(x, o->n_steps, 1);
    if (st == VP_OK) st = vp_nu_session_read(x, volume_out, proj_out, water_out, fat_out, final_loss);
    (void)vp_nu_session_destroy(x);
    return st;
}

extern "C" vp_status vp_tv_grad(const vp_plan* p, const vp_c64* d_vol, float tv_w, float l1_w, float eps,
                                vp_c64* d_grad, int32_t accumulate, void* stream) {
    clear_error();
    if (!p || !d_vol || !d_grad) return fail(VP_ERR_ARG, "vp_tv_grad: NULL argument");
    if (!std::isfinite(tv_w) || !std::isfinite(l1_w) || !(eps > 0) || !std::isfinite(eps))
        return fail(VP_ERR_ARG, "vp_tv_grad: weights must be finite and eps > 0");
    OpScope sc(p, stream);
    vp_status st = sc.begin(false);
    if (st != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.vol[0] = (float2*)d_vol;
    a.one.grad = (float2*)d_grad;
    a.one.tv_w = tv_w;
    a.one.l1_w = l1_w;
    a.one.tv_eps = eps;
    a.accumulate = accumulate != 0;
    a.tasks = sc.t->t_vox;
    a.ntasks = (int)p->t_vox.size();
    hipError_t e = launch_tv_grad(a, sc.s);
    return hip_status(e, "vp_tv_grad");
}

namespace {
__global__ void k_set_counter(int* p, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}
}  // namespace

extern "C" vp_status vp_step(const vp_plan* p, const vp_options* o, const vp_c64* d_vol, const vp_c64* d_grad,
                             vp_c64* d_m, vp_c64* d_v, int64_t t, vp_c64* d_vol_out, void* stream) {
    clear_error();
    if (!p || !o || !d_vol || !d_grad || !d_vol_out) return fail(VP_ERR_ARG, "vp_step: NULL argument");
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    if (o->optimizer == VP_OPT_ADAM && (!d_m || !d_v)) return fail(VP_ERR_ARG, "vp_step: Adam needs d_m and d_v");
    if (t < 1 || t > 0x7fffffff) return fail(VP_ERR_ARG, "vp_step: t must be in [1, 2^31 - 1]");
    const uintptr_t bytes = (uintptr_t)p->voxels() * sizeof(float2);
    const uintptr_t a0 = (uintptr_t)d_vol, b0 = (uintptr_t)d_vol_out;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(VP_ERR_ARG, "vp_step: d_vol_out overlaps d_vol");
    OpScope sc(p, stream);
    if ((st = sc.begin(false)) != VP_OK) return st;
    // the update pass of the current shape, or of four bins per wave where the shape fuses it
    Tiles tl = sc.lay->tiles;
    if (tl.upd_sc == 0) {
        tl.upd_sc = 4;
        tl.gath_res = 0;
        tl.gath_sc = std::min(tl.gath_sc, 16 / tl.gath_rows);
    }
    const Layout* lay = nullptr;
    const DeviceLayout* dl = nullptr;
    if ((st = plan_layout(p, tl, &lay)) != VP_OK || (st = device_layout(p, sc.t, lay, &dl)) != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, lay, dl, &a.one);
    set_hyper(&a.one, o);
    a.one.schedule = VP_SCHED_ALL_BLADES;
    // the pass reads vol[s & 1] and writes vol[(s + 1) & 1] at step counter s = t - 1
    const int s0 = (int)(t - 1);
    a.one.vol[s0 & 1] = (float2*)d_vol;
    a.one.vol[(s0 + 1) & 1] = (float2*)d_vol_out;
    a.one.grad = (float2*)d_grad;
    a.one.m = (float2*)d_m;
    a.one.v = (float2*)d_v;
    a.one.step_limit = 0x7fffffff;
    int* cnt = nullptr;
    hipError_t e = hipMallocAsync((void**)&cnt, 256, sc.s);
    if (e != hipSuccess) return hip_status(e, "vp_step counter");
    hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(64), 0, sc.s, cnt, s0);
    e = hipGetLastError();
    a.one.step = cnt;
    const StageLists L = plan_lists(p, sc.t, lay, dl);
    a.epi = epi_for(o->optimizer, o->tv_weight, o->l1_weight);
    a.stream = stream_for(p->voxels(), o->optimizer);
    a.tasks = L.upd;
    a.ntasks = L.n_upd;
    if (e == hipSuccess) e = launch_update(a, tl.upd_sc, sc.s);
    const hipError_t fe = hipFreeAsync(cnt, sc.s);
    if (e == hipSuccess) e = fe;
    return hip_status(e, "vp_step");
}

extern "C" vp_status vp_render(const vp_plan* p, const vp_c64* d_vol, int32_t split_bin, vp_c64* d_proj,
                               vp_c64* d_water, vp_c64* d_fat, void* stream) {
    clear_error();
    if (!p || !d_vol) return fail(VP_ERR_ARG, "vp_render: NULL argument");
    if (split_bin > p->S) return fail(VP_ERR_ARG, "vp_render: split_bin above n_spec");
    OpScope sc(p, stream);
    vp_status st = sc.begin(false);
    if (st != VP_OK) return st;
    KArgs a{};
    fill_desc(p, sc.t, sc.lay, sc.dl, &a.one);
    a.one.vol[0] = (float2*)d_vol;
    a.split_bin = split_bin;
    a.out0 = (float2*)d_proj;
    a.out1 = (float2*)d_water;
    a.out2 = (float2*)d_fat;
    a.tasks = sc.t->t_render;
    a.ntasks = (int)p->t_render.size();
    return hip_status(launch_render(a, sc.s), "vp_render");
}

// ------------------------------------------------------------------ sessions

vp_session::~vp_session() {
    if (device >= 0) (void)hipSetDevice(device);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (stream) (void)hipStreamSynchronize(stream);
    void* ptrs[] = {vol[0], vol[1], m, v, work, y, loss_part, step_dev, dpart, render, grad};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (h_part) (void)hipHostFree(h_part);
    if (stream && own_stream) (void)hipStreamDestroy(stream);
}

namespace vp {

static bool all_finite(const vp_c64* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i].re) || !std::isfinite(a[i].im)) return false;
    return true;
}

vp_status session_alloc(const vp_plan* p, const vp_options* o, const vp_c64* kspace, const vp_c64* init,
                        hipStream_t stream, vp_session** out, hipStream_t upload, bool wait) {
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    if (!kspace) return fail(VP_ERR_ARG, "session: NULL kspace");
    if (!all_finite(kspace, p->blade_px())) return fail(VP_ERR_NONFINITE, "session: kspace holds NaN or Inf");
    if (init && !all_finite(init, p->voxels())) return fail(VP_ERR_NONFINITE, "session: init holds NaN or Inf");
    std::unique_ptr<vp_session> s(new (std::nothrow) vp_session());
    if (!s) return fail(VP_ERR_NOMEM, "session: out of host memory");
    s->plan = p;
    s->opts = *o;
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    s->device = o->device;
    if (stream) {
        s->stream = stream;
        s->own_stream = false;
    } else {
        e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_status(e, "hipStreamCreate");
        s->own_stream = true;
    }
    st = plan_tables(p, &s->tabs);
    if (st != VP_OK) return st;
    Tiles tl;
    st = tiles_for(p, o, &tl);
    if (st == VP_OK) st = plan_layout(p, tl, &s->layout);
    if (st == VP_OK) st = device_layout(p, s->tabs, s->layout, &s->dlayout);
    if (st != VP_OK) return st;
    const size_t vb = p->voxels() * sizeof(float2);
    const size_t bb = p->blade_px() * sizeof(float2);
#define ALLOC(ptr, bytes)                                               \
    do {                                                                \
        e = hipMalloc((void**)&(ptr), std::max<size_t>(8, (bytes)));   \
        if (e != hipSuccess) return hip_status(e, "session allocation"); \
    } while (0)
    ALLOC(s->vol[0], vb);
    ALLOC(s->vol[1], vb);
    if (o->optimizer == VP_OPT_ADAM) {
        ALLOC(s->m, vb);
        ALLOC(s->v, vb);
    }
    ALLOC(s->work, (size_t)p->nparts * bb);
    ALLOC(s->y, bb);
    ALLOC(s->loss_part, loss_slots(p) * sizeof(float));
    ALLOC(s->step_dev, kCounterBytes);
    ALLOC(s->dpart, 2 * p->t_vox.size() * sizeof(double));
    ALLOC(s->render, 3 * (size_t)p->T * p->n * p->n * sizeof(float2));
#undef ALLOC
    // initial state on `upload` (else the session stream); waited for unless the caller
    // relies on stream order
    hipStream_t us = upload ? upload : s->stream;
    if (init) e = hipMemcpyAsync(s->vol[0], init, vb, hipMemcpyHostToDevice, us);
    else e = hipMemsetAsync(s->vol[0], 0, vb, us);
    if (e == hipSuccess && s->m) e = hipMemsetAsync(s->m, 0, vb, us);
    if (e == hipSuccess && s->v) e = hipMemsetAsync(s->v, 0, vb, us);
    if (e == hipSuccess) e = hipMemcpyAsync(s->y, kspace, bb, hipMemcpyHostToDevice, us);
    if (e == hipSuccess) e = hipMemsetAsync(s->step_dev, 0, kCounterBytes, us);
    if (e == hipSuccess) e = hipMemsetAsync(s->loss_part, 0, loss_slots(p) * sizeof(float), us);
    if (e == hipSuccess && wait) e = hipStreamSynchronize(us);
    if (e != hipSuccess) return hip_status(e, "session upload");
    fill_desc(p, s->tabs, s->layout, s->dlayout, &s->desc);
    set_hyper(&s->desc, o);
    s->desc.vol[0] = s->vol[0];
    s->desc.vol[1] = s->vol[1];
    s->desc.m = s->m;
    s->desc.v = s->v;
    s->desc.work = s->work;
    s->desc.y = s->y;
    s->desc.loss_part = s->loss_part;
    s->desc.step = s->step_dev;
    s->lists = plan_lists(p, s->tabs, s->layout, s->dlayout);
    s->lists.epi = epi_for(o->optimizer, o->tv_weight, o->l1_weight);
    s->lists.stream = stream_for(p->voxels(), o->optimizer);
    if (tl.upd_sc && (st = session_ensure_grad(s.get())) != VP_OK) return st;
    *out = s.release();
    return VP_OK;
}

vp_status session_ensure_grad(vp_session* s) {
    if (s->grad) return VP_OK;
    hipError_t e = hipSetDevice(s->device);
    if (e == hipSuccess) e = hipMalloc((void**)&s->grad, std::max<size_t>(8, s->plan->voxels() * sizeof(float2)));
    if (e != hipSuccess) return hip_status(e, "data gradient allocation");
    s->desc.grad = s->grad;
    return VP_OK;
}

vp_status session_run(vp_session* s, int32_t n_steps, int32_t use_graph) {
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    KArgs a{};
    a.one = s->desc;
    if (use_graph && n_steps > 1) {
        if (!s->gexec) {
            e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_status(e, "hipStreamBeginCapture");
            hipError_t le = hipSuccess;
            launch_step(a, s->lists, s->stream, &le);
            e = hipStreamEndCapture(s->stream, &s->graph);
            if (le != hipSuccess) return hip_status(le, "step capture");
            if (e != hipSuccess) return hip_status(e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&s->gexec, s->graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return hip_status(e, "hipGraphInstantiate");
        }
        for (int i = 0; i < n_steps; ++i) {
            e = hipGraphLaunch(s->gexec, s->stream);
            if (e != hipSuccess) return hip_status(e, "hipGraphLaunch");
        }
    } else {
        for (int i = 0; i < n_steps; ++i) {
            launch_step(a, s->lists, s->stream, &e);
            if (e != hipSuccess) return hip_status(e, "step launch");
        }
    }
    s->steps_done += n_steps;
    return VP_OK;
}

vp_status session_objective(vp_session* s, double* objective, double* data_term) {
    vp_status st = session_objective_enqueue(s, s->stream);
    if (st != VP_OK) return st;
    st = hip_status(hipStreamSynchronize(s->stream), "objective readback");
    if (st != VP_OK) return st;
    return session_objective_finish(s, objective, data_term);
}

vp_status session_objective_enqueue(vp_session* s, hipStream_t stream) {
    const vp_plan* p = s->plan;
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    if (!s->h_part) {
        // pinned, so that the copies below are truly asynchronous
        const size_t bytes = loss_slots(p) * sizeof(float) + 2 * p->t_vox.size() * sizeof(double);
        e = hipHostMalloc((void**)&s->h_part, std::max<size_t>(16, bytes + 8), hipHostMallocDefault);
        if (e != hipSuccess) {
            s->h_part = nullptr;
            return hip_status(e, "objective staging");
        }
    }
    KArgs a{};
    a.one = s->desc;
    a.one.schedule = VP_SCHED_ALL_BLADES;
    a.one.step_limit = 0x7fffffff;
    const StageLists& L = s->lists;
    a.tasks = L.proj; a.ntasks = L.n_proj;
    if ((e = launch_project(a, L.tiles.proj_rows, L.tiles.proj_gw, L.tiles.proj_w, L.re_proj, stream)) != hipSuccess)
        return hip_status(e, "objective");
    a.tasks = L.rows; a.ntasks = L.n_rows;
    if ((e = launch_rows(a, -1, L.fft_n, L.lds_rows, stream)) != hipSuccess) return hip_status(e, "objective");
    a.tasks = L.cols; a.ntasks = L.n_cols; a.mode = COL_STEP;
    if ((e = launch_cols(a, L.fft_n, L.lds_cols, stream)) != hipSuccess) return hip_status(e, "objective");
    a.tasks = L.vox; a.ntasks = L.n_vox; a.dpart = s->dpart;
    if ((e = launch_reg_value(a, stream)) != hipSuccess) return hip_status(e, "objective");
    const size_t nl = loss_slots(p), nd = 2 * p->t_vox.size();
    double* hd = reinterpret_cast<double*>(s->h_part);
    float* hl = reinterpret_cast<float*>(hd + nd);
    e = hipMemcpyAsync(hl, s->loss_part, nl * sizeof(float), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hd, s->dpart, nd * sizeof(double), hipMemcpyDeviceToHost, stream);
    return hip_status(e, "objective readback");
}

vp_status session_objective_finish(vp_session* s, double* objective, double* data_term) {
    const vp_plan* p = s->plan;
    const size_t nl = loss_slots(p), nd = 2 * p->t_vox.size();
    const double* hd = reinterpret_cast<const double*>(s->h_part);
    const float* hl = reinterpret_cast<const float*>(hd + nd);
    double data = 0.0, tv = 0.0, l1 = 0.0;
    for (size_t i = 0; i < nl; ++i) data += (double)hl[i];
    data *= 0.5;
    for (size_t i = 0; i < p->t_vox.size(); ++i) {
        tv += hd[2 * i];
        l1 += hd[2 * i + 1];
    }
    const double obj = data + (double)s->opts.tv_weight * tv + (double)s->opts.l1_weight * l1;
    if (objective) *objective = obj;
    if (data_term) *data_term = data;
    if (!std::isfinite(obj)) return fail(VP_ERR_NONFINITE, "objective is not finite");
    return VP_OK;
}

vp_status session_read(vp_session* s, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out) {
    const vp_plan* p = s->plan;
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    const size_t vb = p->voxels() * sizeof(float2);
    const size_t rb = (size_t)p->T * p->n * p->n * sizeof(float2);
    float2* cur = s->vol[s->steps_done & 1];
    if (proj_out || water_out || fat_out) {
        KArgs a{};
        a.one = s->desc;
        a.split_bin = s->opts.split_bin;
        a.out0 = s->render;
        a.out1 = s->render + (size_t)p->T * p->n * p->n;
        a.out2 = s->render + 2 * (size_t)p->T * p->n * p->n;
        a.tasks = s->lists.render;
        a.ntasks = s->lists.n_render;
        if ((e = launch_render(a, s->stream)) != hipSuccess) return hip_status(e, "render");
        vp_c64* outs[3] = {proj_out, water_out, fat_out};
        for (int i = 0; i < 3 && e == hipSuccess; ++i)
            if (outs[i])
                e = hipMemcpyAsync(outs[i], s->render + (size_t)i * p->T * p->n * p->n, rb, hipMemcpyDeviceToHost,
                                   s->stream);
    }
    if (e == hipSuccess && volume_out) e = hipMemcpyAsync(volume_out, cur, vb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return hip_status(e, "session read");
}

}  // namespace vp

extern "C" vp_status vp_session_create(const vp_plan* p, const vp_options* o, const vp_c64* kspace,
                                       const vp_c64* init, vp_session** out) {
    clear_error();
    if (!p || !o || !out) return fail(VP_ERR_ARG, "vp_session_create: NULL argument");
    return session_alloc(p, o, kspace, init, nullptr, out);
}

extern "C" vp_status vp_session_step(vp_session* s, int32_t n_steps, int32_t use_graph) {
    clear_error();
    if (!s || n_steps < 0) return fail(VP_ERR_ARG, "vp_session_step: bad argument");
    vp_status st = session_run(s, n_steps, use_graph);
    if (st != VP_OK) return st;
    return hip_status(hipStreamSynchronize(s->stream), "vp_session_step");
}

extern "C" vp_status vp_session_steps_done(const vp_session* s, int64_t* steps) {
    if (!s || !steps) return fail(VP_ERR_ARG, "vp_session_steps_done: NULL argument");
    *steps = s->steps_done;
    return VP_OK;
}

extern "C" vp_status vp_session_read(vp_session* s, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out,
                                     vp_c64* fat_out) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_session_read: NULL session");
    return session_read(s, volume_out, proj_out, water_out, fat_out);
}

extern "C" vp_status vp_session_objective(vp_session* s, double* objective, double* data_term) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_session_objective: NULL session");
    return session_objective(s, objective, data_term);
}

extern "C" vp_status vp_session_get_state(vp_session* s, vp_c64* volume, vp_c64* m, vp_c64* v, int64_t* step) {
    clear_error();
    if (!s) return fail(VP_ERR_ARG, "vp_session_get_state: NULL session");
    const vp_plan* p = s->plan;
    hipError_t e = hipSetDevice(s->device);
    const size_t vb = p->voxels() * sizeof(float2);
    if (e == hipSuccess && volume)
        e = hipMemcpyAsync(volume, s->vol[s->steps_done & 1], vb, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && m) {
        if (s->m) e = hipMemcpyAsync(m, s->m, vb, hipMemcpyDeviceToHost, s->stream);
        else std::memset(m, 0, vb);
    }
    if (e == hipSuccess && v) {
        if (s->v) e = hipMemcpyAsync(v, s->v, vb, hipMemcpyDeviceToHost, s->stream);
        else std::memset(v, 0, vb);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (step) *step = s->steps_done;
    return hip_status(e, "vp_session_get_state");
}

extern "C" vp_status vp_session_set_state(vp_session* s, const vp_c64* volume, const vp_c64* m, const vp_c64* v,
                                          int64_t step) {
    clear_error();
    if (!s || !volume || step < 0 || step > 0x7ffffffe) return fail(VP_ERR_ARG, "vp_session_set_state: bad argument");
    const vp_plan* p = s->plan;
    if (!all_finite(volume, p->voxels())) return fail(VP_ERR_NONFINITE, "vp_session_set_state: non-finite volume");
    hipError_t e = hipSetDevice(s->device);
    const size_t vb = p->voxels() * sizeof(float2);
    const int st32 = (int)step;
    if (e == hipSuccess) e = hipMemcpyAsync(s->vol[step & 1], volume, vb, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && s->m) {
        if (m) e = hipMemcpyAsync(s->m, m, vb, hipMemcpyHostToDevice, s->stream);
        else e = hipMemsetAsync(s->m, 0, vb, s->stream);
    }
    if (e == hipSuccess && s->v) {
        if (v) e = hipMemcpyAsync(s->v, v, vb, hipMemcpyHostToDevice, s->stream);
        else e = hipMemsetAsync(s->v, 0, vb, s->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s->step_dev, &st32, sizeof st32, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) s->steps_done = step;
    return hip_status(e, "vp_session_set_state");
}

extern "C" vp_status vp_session_stage_times(vp_session* s, int32_t n_steps, double* stage_ms) {
    clear_error();
    if (!s || !stage_ms || n_steps < 1 || n_steps > 100000)
        return fail(VP_ERR_ARG, "vp_session_stage_times: bad argument");
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    const int ne = (kStages + 1) * n_steps;
    std::vector<hipEvent_t> ev(ne, nullptr);
    vp_status st = VP_OK;
    for (int i = 0; i < ne && st == VP_OK; ++i) st = hip_status(hipEventCreate(&ev[i]), "hipEventCreate");
    KArgs a{};
    a.one = s->desc;
    for (int k = 0; k < n_steps && st == VP_OK; ++k) {
        launch_step(a, s->lists, s->stream, &e, &ev[(size_t)k * (kStages + 1)]);
        st = hip_status(e, "stage-timed step");
        if (st == VP_OK) ++s->steps_done;
    }
    if (st == VP_OK) st = hip_status(hipStreamSynchronize(s->stream), "stage-timed steps");
    for (int j = 0; j < kStages; ++j) stage_ms[j] = 0.0;
    for (int k = 0; k < n_steps && st == VP_OK; ++k)
        for (int j = 0; j < kStages && st == VP_OK; ++j) {
            float ms = 0.f;
            hipEvent_t* b = &ev[(size_t)k * (kStages + 1)];
            st = hip_status(hipEventElapsedTime(&ms, b[j], b[j + 1]), "hipEventElapsedTime");
            stage_ms[j] += ms / n_steps;
        }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    return st;
}

extern "C" vp_status vp_session_destroy(vp_session* s) {
    delete s;
    return VP_OK;
}

// ------------------------------------------------------------------ whole reconstructions

extern "C" vp_status vp_reconstruct(const vp_plan* p, const vp_options* o, const vp_c64* kspace, const vp_c64* init,
                                    vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out,
                                    double* final_loss) {
    clear_error();
    if (!p || !o || !kspace) return fail(VP_ERR_ARG, "vp_reconstruct: NULL argument");
    vp_session* raw = nullptr;
    vp_status st = session_alloc(p, o, kspace, init, nullptr, &raw);
    if (st != VP_OK) return st;
    std::unique_ptr<vp_session> s(raw);
    st = session_run(s.get(), o->n_steps, 1);
    if (st != VP_OK) return st;
    double obj = 0.0;
    st = session_objective(s.get(), &obj, nullptr);
    if (final_loss) *final_loss = obj;
    const vp_status rs = session_read(s.get(), volume_out, proj_out, water_out, fat_out);
    if (st != VP_OK) return st;
    return rs;
}
