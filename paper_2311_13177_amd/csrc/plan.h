// Host-side plan of libvp: validated geometry, FP64-derived tables and launch lists.
#pragma once

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "vp.h"
#include "vp_internal.h"

namespace vp {

// Sets the thread-local error message and returns `code`.
vp_status fail(vp_status code, const char* fmt, ...);
void clear_error();

// Tile shape of the projection and gather work items (see vp_internal.h). Results never
// depend on it: only the work decomposition changes.
struct Tiles {
    int proj_rows = 2, proj_gw = 1, gath_rows = 2, gath_sc = 1;
    int upd_sc = 0;  // 0: update fused into the gather; else bins per wave of the update pass
    int gath_w = 4;  // waves per gather item
    int proj_w = 4;  // waves per projection item
    int gath_res = 0;  // 1: the resident-parts gather (every part of a knot staged at once)
    int key() const {
        return proj_rows | proj_gw << 4 | gath_rows << 8 | gath_sc << 12 | upd_sc << 16 | gath_w << 20 | proj_w << 24 |
               gath_res << 28;
    }
    bool operator==(const Tiles& o) const { return key() == o.key(); }
};

// Projection groups and work lists of one tile shape.
struct Layout {
    Tiles tiles;
    std::vector<ProjGroup> groups;
    std::vector<Task> t_proj, t_gath, t_upd;
    int re_proj = 0, re_gath = 0;  // largest staged region (elements) of an item
    size_t lds_res = 0;            // resident-parts gather: LDS bytes of the largest knot
};

// A layout's tables on one device.
struct DeviceLayout {
    ProjGroup* groups = nullptr;
    Task* t_proj = nullptr;
    Task* t_gath = nullptr;
    Task* t_upd = nullptr;
    ~DeviceLayout();
};

// Per-device copies of a plan's constant tables and work lists.
struct DeviceTables {
    int device = -1;
    uint8_t* mask = nullptr;
    ShearEntry* shear = nullptr;
    BladeDev* blade = nullptr;
    int* knot_ptr = nullptr;
    KnotEntry* knot_ent = nullptr;
    ShearEntry* knot_tap = nullptr;
    KnotInfo* knots = nullptr;
    float2* tw = nullptr;
    Task* t_rows = nullptr;
    Task* t_cols = nullptr;
    Task* t_vox = nullptr;
    Task* t_render = nullptr;
    std::map<int, std::unique_ptr<DeviceLayout>> layouts;  // by Tiles::key()
    // blade-aligned sampling tables (uploaded on first use)
    int* nu_lines = nullptr;
    double2* nu_cs = nullptr;
    float2* nu_ph = nullptr;
    float* nu_dea = nullptr;
    float* nu_kb = nullptr;
    Task* nu_rows = nullptr;
    ~DeviceTables();
};

// Host tables of blade-aligned sampling (see the blade-sampling kernels).
struct NuHost {
    int lmax = 0;
    float kmax = 0.f;
    std::vector<int> lines;
    std::vector<double2> cs;         // [B]
    std::vector<float2> ph;          // [B][lmax][n]
    std::vector<float> dea, kb;      // [n], [kNuTable + 1]
    std::vector<Task> rows;          // row-pass tasks of the oversampled plan that touch the image's rows
};

}  // namespace vp

struct vp_plan {
    int n = 0, S = 0, T = 0, B = 0;
    std::vector<double> angle, tau, shift;
    std::vector<int> lines;
    std::vector<uint8_t> mask;           // [B][n][n]
    std::vector<vp::ShearEntry> shear;   // [B][S]
    std::vector<float> fx, fy;           // [B][S] fractional parts, for inspection
    std::vector<vp::BladeDev> blade;     // [B]
    std::vector<float> alpha;            // [B]
    std::vector<int> knot_ptr;           // [T+1]
    std::vector<vp::KnotEntry> knot_ent;
    std::vector<vp::ShearEntry> knot_tap;  // [entries][S]: the blade's taps times the entry weight
    std::vector<vp::KnotInfo> knots;    // [T]
    int max_knot_parts = 0;              // most blade parts feeding one knot
    std::vector<float2> tw;              // [n]
    int nstage = 0;
    int radix[vp::kMaxStages] = {0};
    int nparts = 1;
    int n_col_items = 0;
    // Work lists of the tile-independent stages (slice index 0; batches rebase it).
    std::vector<vp::Task> t_rows, t_cols, t_vox, t_render;
    // Dynamic LDS bytes per kernel.
    size_t lds_rows = 0, lds_cols = 0;
    // The layout of the default tile shape, built and checked at creation.
    vp::Tiles base_tiles;

    mutable std::mutex mu;
    mutable std::map<int, std::unique_ptr<vp::Layout>> layouts;  // host layouts by Tiles::key()
    mutable std::map<int, std::unique_ptr<vp::DeviceTables>> dev;
    // The same geometry with a knot per blade (built on first use; K-Planes fits).
    mutable std::mutex mu_derived;
    mutable std::unique_ptr<vp_plan> per_blade;
    // Blade-aligned sampling: its host tables and the plan of the oversampled grid
    // (2n x 2n, the same blades; its DFT passes only), built on first use.
    mutable std::unique_ptr<vp::NuHost> nu_host;
    mutable std::unique_ptr<vp_plan> over;

    uint64_t voxels() const { return (uint64_t)T * S * n * n; }
    uint64_t blade_px() const { return (uint64_t)B * n * n; }
};

namespace vp {

// The plan's geometry with one knot per blade (knot b holds blade b with weight 1, one
// work part per blade), built on first use and kept with the plan.
vp_status plan_per_blade(const vp_plan* plan, const vp_plan** out);
// Blade-aligned sampling: host tables and the oversampled grid's plan (VP_ERR_UNSUPPORTED
// if 2n exceeds the largest transform length).
vp_status plan_nu(const vp_plan* plan, const NuHost** host, const vp_plan** over);
// The tables of plan_nu on the device of `t`, uploaded on first use.
vp_status nu_tables(const vp_plan* plan, const NuHost* host, DeviceTables* t);

// Device tables of `plan` on the current device, uploading them on first use.
vp_status plan_tables(const vp_plan* plan, DeviceTables** out);

// Host layout of `plan` for tile shape `t` (built on first use and kept with the plan).
// VP_ERR_UNSUPPORTED if the shape is not compiled or a staged region would not fit.
vp_status plan_layout(const vp_plan* plan, const Tiles& t, const Layout** out);
// A layout's tables on the device of `tabs`, uploaded on first use.
vp_status device_layout(const vp_plan* plan, DeviceTables* tabs, const Layout* L, const DeviceLayout** out);
// Tile shape chosen without measuring, from the plan's sizes.
Tiles heuristic_tiles(const vp_plan* plan);

// Fills the plan-constant part of a slice descriptor from device tables and a layout.
void fill_desc(const vp_plan* plan, const DeviceTables* t, const Layout* L, const DeviceLayout* dl, SliceDesc* d);

// Loss partial slots (floats) per reconstruction.
inline uint64_t loss_slots(const vp_plan* p) { return (uint64_t)p->B * p->n_col_items; }

}  // namespace vp
