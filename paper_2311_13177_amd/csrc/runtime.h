// Internal declarations shared by the runtime, batch and server translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "plan.h"

namespace vp {

// Kernel launchers (kernels.hip).
// re: largest staged region (elements) over the work items' slices.
// waves: 4 or 8 per work item (the layout's proj_w: its groups hold waves * gw parts)
hipError_t launch_project(const KArgs& a, int rows, int gw, int waves, int re, hipStream_t s);
// n: the common length of every slice of the launch (0 if they differ).
hipError_t launch_rows(const KArgs& a, int dir, int n, size_t lds, hipStream_t s);
hipError_t launch_cols(const KArgs& a, int n, size_t lds, hipStream_t s);
// waves: 4 or 8 per work item (the layout's gath_w: its bin chunks hold waves * sc bins)
hipError_t launch_gather(const KArgs& a, int mode, int rows, int sc, int waves, int re, hipStream_t s);
// The resident-parts gather: lds bytes of the largest knot's parts (Layout::lds_res).
// re: largest staged region (elements) of the layout (re_gath).
hipError_t launch_gather_res(const KArgs& a, int mode, int rows, int sc, int waves, int re, size_t lds, hipStream_t s);
hipError_t launch_update(const KArgs& a, int sc, hipStream_t s);
hipError_t launch_tv_grad(const KArgs& a, hipStream_t s);
hipError_t launch_reg_value(const KArgs& a, hipStream_t s);
hipError_t launch_render(const KArgs& a, hipStream_t s);
hipError_t launch_baseline_avg(const uint8_t* mask, const float2* y, float2* out, int n, int window, int first,
                               int n_frames, hipStream_t s);
hipError_t launch_psnr(const float2* img, const float2* truth, long long npx, int n_images, double* terms,
                       hipStream_t s);

// Device work lists of one optimiser step and the dynamic LDS of each stage.
struct StageLists {
    const Task* proj = nullptr;
    const Task* rows = nullptr;
    const Task* cols = nullptr;
    const Task* gath = nullptr;
    const Task* vox = nullptr;
    const Task* render = nullptr;
    const Task* upd = nullptr;
    int n_slices = 1;  // slices whose step counters the step advances
    int n_proj = 0, n_rows = 0, n_cols = 0, n_gath = 0, n_vox = 0, n_render = 0, n_upd = 0;
    Tiles tiles;
    int fft_n = 0;  // common length of every slice (0 if they differ)
    size_t lds_rows = 0, lds_cols = 0;
    int re_proj = 0, re_gath = 0;  // largest staged regions (elements)
    size_t lds_res = 0;            // resident-parts gather: LDS bytes of the largest knot
    int epi = EPI_GENERIC;         // optimiser epilogue every slice of the step can take
    int stream = 0;                // the step's state exceeds kStreamState (EPI_STREAM)
};

StageLists plan_lists(const vp_plan* p, const DeviceTables* t, const Layout* L, const DeviceLayout* dl);
// Whether a step over `voxels` voxels (summed over its slices) streams its state.
inline int stream_for(uint64_t voxels, int optimizer) {
    return voxels * sizeof(float2) * (optimizer == VP_OPT_ADAM ? 4u : 2u) > kStreamState ? 1 : 0;
}
// The gather of a step's layout (resident-parts or staged a few parts at a time).
hipError_t launch_gather_lists(const KArgs& a, int mode, const StageLists& L, hipStream_t s);
// Tile shape for a plan under options: explicit tiles from the options, else the tuned
// shape recorded for this plan's sizes on the device (tuning first when the options ask
// for it and none is recorded), else the plan's heuristic shape.
vp_status tiles_for(const vp_plan* p, const vp_options* o, Tiles* out);
// Tuned shape recorded for the plan's sizes on `device`, if any.
bool tuned_tiles(const vp_plan* p, int device, int optimizer, Tiles* out);
// Measures the candidate tile shapes on the current device and records the fastest.
vp_status tune_plan(const vp_plan* p, const vp_options* o, Tiles* out);
// Enqueues one optimiser step (project, row DFT, column pass, inverse row DFT,
// gather + update, the last also advancing the step counters) for the descriptors
// `base` refers to.
// With `ev` (kStages + 1 events) an event is recorded before each stage and after the last.
void launch_step(const KArgs& base, const StageLists& L, hipStream_t s, hipError_t* err, hipEvent_t* ev = nullptr);
constexpr int kStages = 5;
// Per-slice device counter block: the step counter (int at offset 0) and its snapshot
// (int kSnapWord).
constexpr size_t kCounterBytes = 256;
static_assert(kCounterBytes >= (kSnapWord + 1) * sizeof(int), "counter block holds the snapshot");

vp_status hip_status(hipError_t e, const char* what);
vp_status check_options(const vp_plan* p, const vp_options* o);

}  // namespace vp

struct vp_session {
    const vp_plan* plan = nullptr;
    vp_options opts{};
    int device = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    vp::DeviceTables* tabs = nullptr;
    const vp::Layout* layout = nullptr;
    const vp::DeviceLayout* dlayout = nullptr;
    float2* vol[2] = {nullptr, nullptr};
    float2* m = nullptr;
    float2* v = nullptr;
    float2* work = nullptr;
    float2* y = nullptr;
    float* loss_part = nullptr;
    int* step_dev = nullptr;
    double* dpart = nullptr;
    float2* render = nullptr;
    float2* grad = nullptr;  // data gradient, allocated when a separate update pass runs
    void* h_part = nullptr;  // pinned objective partials (doubles, then loss floats)
    int64_t steps_done = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    vp::SliceDesc desc{};
    vp::StageLists lists{};
    ~vp_session();
};

namespace vp {

// Device-resident group of slices sharing one stream: descriptors, concatenated work
// lists and (optionally) a captured step. Used by batched reconstructions and the server.
struct SliceGroup {
    int device = -1;
    hipStream_t stream = nullptr;
    SliceDesc* d_descs = nullptr;
    Task* d_tasks = nullptr;
    size_t cap_descs = 0, cap_tasks = 0;  // device capacities (grow only)
    std::vector<SliceDesc> h_descs;       // host copies, kept until the stream has read them
    std::vector<Task> h_tasks;
    StageLists lists{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    ~SliceGroup();
    void drop_graph();
};
// Builds descriptors and concatenated work lists for `sessions` (slice i = sessions[i],
// stopping at limits[i] steps) and enqueues their upload on the group's stream (no
// wait); drops any captured graph. Call it only once the stream has passed the previous
// upload (the host copies are reused).
vp_status group_build(SliceGroup* g, const std::vector<vp_session*>& sessions, const std::vector<int>& limits);
// Enqueues n_steps steps of every slice of the group (use_graph: capture one step once).
vp_status group_run(SliceGroup* g, int n_steps, bool use_graph);

// Allocates and uploads a session on `stream` (nullptr: a stream of its own). The initial
// state is enqueued on `upload` (nullptr: the session stream) and waited for if `wait`;
// otherwise the caller keeps kspace and init alive until that stream has passed them.
vp_status session_alloc(const vp_plan* p, const vp_options* o, const vp_c64* kspace, const vp_c64* init,
                        hipStream_t stream, vp_session** out, hipStream_t upload = nullptr, bool wait = true);
vp_status session_run(vp_session* s, int32_t n_steps, int32_t use_graph);
// Allocates the session's data-gradient buffer (for a separate update pass) if missing.
vp_status session_ensure_grad(vp_session* s);
vp_status session_objective(vp_session* s, double* objective, double* data_term);
// The objective in two halves: kernels and pinned read-back enqueued on `stream`, then
// (after the caller has synchronised that stream) the host reduction.
vp_status session_objective_enqueue(vp_session* s, hipStream_t stream);
vp_status session_objective_finish(vp_session* s, double* objective, double* data_term);
vp_status session_read(vp_session* s, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out);
}  // namespace vp
