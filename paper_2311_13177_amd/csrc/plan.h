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

// Per-device copies of a plan's constant tables and work lists.
struct DeviceTables {
    int device = -1;
    uint8_t* mask = nullptr;
    ShearEntry* shear = nullptr;
    BladeDev* blade = nullptr;
    int* knot_ptr = nullptr;
    KnotEntry* knot_ent = nullptr;
    ProjGroup* groups = nullptr;
    KnotInfo* knots = nullptr;
    float2* tw = nullptr;
    Task* t_proj = nullptr;
    Task* t_rows = nullptr;
    Task* t_cols = nullptr;
    Task* t_gath = nullptr;
    Task* t_vox = nullptr;
    Task* t_render = nullptr;
    ~DeviceTables();
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
    std::vector<vp::ProjGroup> groups;
    std::vector<vp::KnotInfo> knots;    // [T]
    int proj_gw = 1;                     // blade parts per wave in a projection item
    int gath_sc = 1;                     // bins per wave in a gather item
    std::vector<float2> tw;              // [n]
    int nstage = 0;
    int radix[vp::kMaxStages] = {0};
    int nparts = 1;
    int n_col_items = 0;
    // Work lists (slice index 0; batches rebase it).
    std::vector<vp::Task> t_proj, t_rows, t_cols, t_gath, t_vox, t_render;
    // Dynamic LDS bytes per kernel.
    size_t lds_rows = 0, lds_cols = 0;
    // Largest staged region (elements) of a projection / gather work item.
    int re_proj = 0, re_gath = 0;

    mutable std::mutex mu;
    mutable std::map<int, std::unique_ptr<vp::DeviceTables>> dev;

    uint64_t voxels() const { return (uint64_t)T * S * n * n; }
    uint64_t blade_px() const { return (uint64_t)B * n * n; }
};

namespace vp {

// Device tables of `plan` on the current device, uploading them on first use.
vp_status plan_tables(const vp_plan* plan, DeviceTables** out);

// Fills the plan-constant part of a slice descriptor from device tables.
void fill_desc(const vp_plan* plan, const DeviceTables* t, SliceDesc* d);

// Loss partial slots (floats) per reconstruction.
inline uint64_t loss_slots(const vp_plan* p) { return (uint64_t)p->B * p->n_col_items; }

}  // namespace vp
