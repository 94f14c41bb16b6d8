// Tile-shape autotuner of libvp: times the compiled projection and gather tile shapes
// that fit a plan on the device and records the fastest per plan sizes. The shape only
// changes how the work is cut into work items (every shape gives the same bits), so the
// choice is purely a matter of speed.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "plan.h"
#include "runtime.h"

namespace vp {
namespace {

// What decides the fastest shape: sizes, the staged halo, the parts feeding a knot and
// the epilogue (Adam or GD). Plans with equal keys share a tuned shape.
struct TuneKey {
    int device, n, S, T, B, nparts, max_parts, hx, hy, optimizer;
    bool operator<(const TuneKey& o) const {
        return std::tie(device, n, S, T, B, nparts, max_parts, hx, hy, optimizer) <
               std::tie(o.device, o.n, o.S, o.T, o.B, o.nparts, o.max_parts, o.hx, o.hy, o.optimizer);
    }
};

std::mutex g_mu;
std::map<TuneKey, Tiles> g_tuned;

TuneKey key_of(const vp_plan* p, int device, int optimizer) {
    int hx = 0, hy = 0;
    for (const KnotInfo& k : p->knots) {
        hx = std::max(hx, k.ox_max - k.ox_min);
        hy = std::max(hy, k.oy_max - k.oy_min);
    }
    return TuneKey{device, p->n, p->S, p->T, p->B, p->nparts, p->max_knot_parts, hx, hy, optimizer};
}

int pow2_at_least(int v) {
    int r = 1;
    while (r < v) r <<= 1;
    return r;
}

// Mean duration (ms) of `reps` launches after one untimed launch.
template <class F>
vp_status time_launches(hipStream_t s, int reps, F launch, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e == hipSuccess) *ms /= (float)reps;
    return hip_status(e, "autotune timing");
}

constexpr int kReps = 5;

}  // namespace

bool tuned_tiles(const vp_plan* p, int device, int optimizer, Tiles* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tuned.find(key_of(p, device, optimizer));
    if (it == g_tuned.end()) return false;
    *out = it->second;
    return true;
}

vp_status tiles_for(const vp_plan* p, const vp_options* o, Tiles* out) {
    const vp_tiles& t = o->tiles;
    if (t.proj_rows || t.proj_parts || t.gath_rows || t.gath_bins || t.upd_bins || t.gath_waves || t.proj_waves ||
        t.gath_resident) {
        *out = Tiles{t.proj_rows, t.proj_parts, t.gath_rows, t.gath_bins, t.upd_bins,
                     t.gath_waves ? t.gath_waves : 4, t.proj_waves ? t.proj_waves : 4, t.gath_resident};
        return VP_OK;
    }
    if (tuned_tiles(p, o->device, o->optimizer, out)) return VP_OK;
    if (o->autotune) return tune_plan(p, o, out);
    *out = p->base_tiles;
    return VP_OK;
}

vp_status tune_plan(const vp_plan* p, const vp_options* o, Tiles* out) {
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    // scratch reconstruction state on the plan's built-in shape, zero measurements
    std::vector<vp_c64> zeros;
    try {
        zeros.assign(p->blade_px(), vp_c64{0.f, 0.f});
    } catch (const std::bad_alloc&) {
        return fail(VP_ERR_NOMEM, "autotune: out of host memory");
    }
    vp_options so = *o;
    so.tiles = vp_tiles{p->base_tiles.proj_rows, p->base_tiles.proj_gw, p->base_tiles.gath_rows,
                        p->base_tiles.gath_sc, 0, p->base_tiles.gath_w, p->base_tiles.proj_w,
                        p->base_tiles.gath_res};
    so.autotune = 0;
    vp_session* raw = nullptr;
    st = session_alloc(p, &so, zeros.data(), nullptr, nullptr, &raw);
    if (st != VP_OK) return st;
    std::unique_ptr<vp_session> s(raw);
    DeviceTables* tabs = s->tabs;

    Tiles best = p->base_tiles;
    best.upd_sc = 0;
    // projection: every compiled (rows, parts per wave) with four and with eight waves per
    // item that keeps every wave busy (eight only where a knot has more than four parts)
    float best_ms = FLT_MAX;
    for (int waves = 4; waves <= 8; waves += 4) {
        if (waves == 8 && p->max_knot_parts <= 4) break;
        const int gw_cap = std::min(8, pow2_at_least((std::max(1, p->max_knot_parts) + waves - 1) / waves));
        for (int rows : {1, 2, 4, 8, 12}) {
            for (int gw = 1; gw <= gw_cap; gw *= 2) {
                if (!proj_tiles_ok(rows, gw)) continue;
                Tiles t = p->base_tiles;
                t.proj_rows = rows;
                t.proj_gw = gw;
                t.proj_w = waves;
                const Layout* L = nullptr;
                const DeviceLayout* dl = nullptr;
                if (plan_layout(p, t, &L) != VP_OK) {
                    clear_error();
                    continue;
                }
                if ((st = device_layout(p, tabs, L, &dl)) != VP_OK) return st;
                KArgs a{};
                a.one = s->desc;
                a.one.groups = dl->groups;
                a.tasks = dl->t_proj;
                a.ntasks = (int)L->t_proj.size();
                float ms = 0.f;
                st = time_launches(
                    s->stream, kReps,
                    [&] { return launch_project(a, rows, gw, waves, L->re_proj, s->stream); }, &ms);
                if (st != VP_OK) return st;
                if (ms < best_ms) {
                    best_ms = ms;
                    best.proj_rows = rows;
                    best.proj_gw = gw;
                    best.proj_w = waves;
                }
            }
        }
    }
    // gather: every compiled (rows, bins per wave) with four and with eight waves per item
    // that keeps every wave busy, with the update fused (mode GATHER_STEP) and storing the
    // data gradient for a separate update pass (GATHER_STORE); then every update-pass shape
    if ((st = session_ensure_grad(s.get())) != VP_OK) return st;
    float fused_ms = FLT_MAX, store_ms = FLT_MAX, upd_ms = FLT_MAX;
    Tiles fused = best, split = best;
    // (the fused update also with every part of a knot resident, where the layout allows it)
    for (int mode = GATHER_STORE; mode <= GATHER_STEP; ++mode) {
        for (int res = 0; res <= (mode == GATHER_STEP ? 1 : 0); ++res) {
            for (int waves = 4; waves <= 8; waves += 4) {
                // bins per wave up to the first power of two that covers S with every wave
                const int sc_cap = std::min(8, pow2_at_least((p->S + waves - 1) / waves));
                for (int rows = 2; rows <= 4; rows *= 2) {
                    for (int sc = 1; sc <= sc_cap; sc *= 2) {
                        if (!gath_tiles_ok(rows, sc, res == 1)) continue;
                        Tiles t = p->base_tiles;
                        t.gath_rows = rows;
                        t.gath_sc = sc;
                        t.gath_w = waves;
                        t.upd_sc = 0;
                        t.gath_res = res;
                        const Layout* L = nullptr;
                        const DeviceLayout* dl = nullptr;
                        if (plan_layout(p, t, &L) != VP_OK) {
                            clear_error();
                            continue;
                        }
                        if ((st = device_layout(p, tabs, L, &dl)) != VP_OK) return st;
                        KArgs a{};
                        a.one = s->desc;
                        a.epi = s->lists.epi;
                        a.stream = s->lists.stream;
                        a.tasks = dl->t_gath;
                        a.ntasks = (int)L->t_gath.size();
                        float ms = 0.f;
                        st = time_launches(
                            s->stream, kReps,
                            [&] {
                                return res ? launch_gather_res(a, mode, rows, sc, waves, L->re_gath, L->lds_res, s->stream)
                                           : launch_gather(a, mode, rows, sc, waves, L->re_gath, s->stream);
                            },
                            &ms);
                        if (st != VP_OK) return st;
                        float& bm = mode == GATHER_STEP ? fused_ms : store_ms;
                        Tiles& bt = mode == GATHER_STEP ? fused : split;
                        if (ms < bm) {
                            bm = ms;
                            bt.gath_rows = rows;
                            bt.gath_sc = sc;
                            bt.gath_w = waves;
                            bt.gath_res = res;
                        }
                    }
                }
            }
        }
    }
    for (int usc = 2; usc <= 8; usc *= 2) {
        Tiles t = p->base_tiles;
        t.upd_sc = usc;
        t.gath_res = 0;
        t.gath_sc = std::min(t.gath_sc, 16 / t.gath_rows);
        const Layout* L = nullptr;
        const DeviceLayout* dl = nullptr;
        if (plan_layout(p, t, &L) != VP_OK) {
            clear_error();
            continue;
        }
        if ((st = device_layout(p, tabs, L, &dl)) != VP_OK) return st;
        KArgs a{};
        a.one = s->desc;
        a.epi = s->lists.epi;
        a.stream = s->lists.stream;
        a.tasks = dl->t_upd;
        a.ntasks = (int)L->t_upd.size();
        float ms = 0.f;
        st = time_launches(s->stream, kReps, [&] { return launch_update(a, usc, s->stream); }, &ms);
        if (st != VP_OK) return st;
        if (ms < upd_ms) {
            upd_ms = ms;
            split.upd_sc = usc;
        }
    }
    if (store_ms + upd_ms < fused_ms) {
        best.gath_rows = split.gath_rows;
        best.gath_sc = split.gath_sc;
        best.gath_w = split.gath_w;
        best.upd_sc = split.upd_sc;
        best.gath_res = 0;
    } else {
        best.gath_rows = fused.gath_rows;
        best.gath_sc = fused.gath_sc;
        best.gath_w = fused.gath_w;
        best.upd_sc = 0;
        best.gath_res = fused.gath_res;
    }
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return hip_status(e, "autotune");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_tuned[key_of(p, o->device, o->optimizer)] = best;
    }
    *out = best;
    return VP_OK;
}

}  // namespace vp

using namespace vp;

static vp_tiles to_abi(const Tiles& t) {
    return vp_tiles{t.proj_rows, t.proj_gw, t.gath_rows, t.gath_sc, t.upd_sc, t.gath_w, t.proj_w, t.gath_res};
}

extern "C" vp_status vp_plan_tune(const vp_plan* p, const vp_options* o, vp_tiles* out) {
    clear_error();
    if (!p || !o || !out) return fail(VP_ERR_ARG, "vp_plan_tune: NULL argument");
    Tiles t;
    const vp_status st = tune_plan(p, o, &t);
    if (st == VP_OK) *out = to_abi(t);
    return st;
}

extern "C" vp_status vp_plan_tiles(const vp_plan* p, const vp_options* o, vp_tiles* out) {
    clear_error();
    if (!p || !o || !out) return fail(VP_ERR_ARG, "vp_plan_tiles: NULL argument");
    vp_status st = check_options(p, o);
    if (st != VP_OK) return st;
    Tiles t;
    st = tiles_for(p, o, &t);
    if (st != VP_OK) return st;
    const Layout* L = nullptr;
    st = plan_layout(p, t, &L);
    if (st == VP_OK) *out = to_abi(t);
    return st;
}
