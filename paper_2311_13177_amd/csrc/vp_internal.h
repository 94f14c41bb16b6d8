// Internal types shared by the host plan/runtime and the HIP kernels of libvp.
//
// Device data layout (all complex values are float2 = (re, im)):
//   volume      [T][S][n][n]   two copies (ping-pong by step parity) during a fit
//   Adam m, v   [T][S][n][n]   float2 per voxel: moments of Re and of Im
//   blade work  [B][P][n][n]   P = 1 (static) or 2 (dynamic: the unweighted
//                              projections of a blade's two knots); part 0 also
//                              carries the blade image through the FFT passes
//   measured y  [B][n][n]      unshifted k-space
//   mask        [B][n][n]      uint8
#pragma once

#include <cstdint>
#include <hip/hip_runtime.h>

namespace vp {

constexpr int kMaxN = 512;
constexpr int kMaxS = 256;
constexpr int kMaxT = 64;
constexpr int kMaxB = 256;
constexpr int kMaxStages = 12;
constexpr double kMaxShift = 16.0;
constexpr int kThreads = 256;

// Projection and gather tiles: 64 columns (one per lane of a wave) by a per-layout
// number of rows. A projection work item covers one tile for a group of up to 4 * GW
// blade parts of one knot (parts dealt round-robin to the block's four waves); a gather
// work item covers one tile for 4 * SC spectral bins (SC consecutive bins per wave).
// Rows, GW and SC are template parameters of the kernels; these are the compiled
// combinations (at most 16 accumulators per lane).
constexpr int kTileW = 64;
constexpr int kXcds = 8;  // accelerator complex dies, each with its own L2
__host__ __device__ constexpr bool pow2_le(int v, int hi) { return v >= 1 && v <= hi && (v & (v - 1)) == 0; }
// (Twelve-row projection tiles too, one part per wave: at n = 192 they make exactly one
// round of items on the chip.)
__host__ __device__ constexpr bool proj_tiles_ok(int rows, int gw) {
    return (pow2_le(rows, 8) || (rows == 12 && gw == 1)) && pow2_le(gw, 8) && rows * gw <= 16;
}
// (The resident-parts gather keeps one bin's sums at a time, so it also takes 4 x 8.)
__host__ __device__ constexpr bool gath_tiles_ok(int rows, int sc, bool resident = false) {
    return pow2_le(rows, 4) && rows >= 2 && pow2_le(sc, 8) && (resident || rows * sc <= 16);
}
// Waves per projection or gather item (the waves share the item's staged regions).
__host__ __device__ constexpr bool item_waves_ok(int w) { return w == 4 || w == 8; }
// The optimiser update runs fused into the gather (0) or as a separate pass over the
// stored data gradient with 2, 4 or 8 bins per wave.
__host__ __device__ constexpr bool upd_tiles_ok(int sc) { return sc == 0 || sc == 2 || sc == 4 || sc == 8; }
// Resident-parts gather (tile field gath_res): every blade part of a knot is staged at
// once. A layout may take it where each knot's region is at most kResRegion elements, it
// has at most kResMaxParts parts, and all of them fit kResLds bytes of LDS.
constexpr int kResRegion = 2048;
constexpr int kResMaxParts = 32;
constexpr size_t kResLds = 65536;
// Staged region elements per thread (register prefetch depth of the LDS staging).
constexpr int kStageMax = 16;
// A staged region of re elements (re <= kStageMax * kThreads) is loaded several planes
// (bins or blade images) per barrier phase so that many loads are in flight: three
// planes of up to 5 elements per thread, two of up to 8, or one of up to 16. The LDS
// holds two phases (double buffering).
__host__ __device__ constexpr int stage_planes(int re) {
    return re <= 5 * kThreads ? 3 : (re <= 8 * kThreads ? 2 : 1);
}
__host__ __device__ constexpr int stage_depth(int re) {
    return re <= 5 * kThreads ? 5 : (re <= 8 * kThreads ? 8 : 16);
}
__host__ __device__ constexpr size_t stage_lds_bytes(int re) {
    return 2 * (size_t)stage_planes(re) * (size_t)re * 8;
}
// Voxel-wise kernels (TV, render, objective): elements per work item.
constexpr int kVoxItem = 4096;

// Rows per row-FFT work item and columns per column-FFT work item, as functions of n
// only (each transform is independent, so they never change a result): small enough
// items that a blade set spreads over the whole chip.
__host__ __device__ constexpr int fft_rows_per_item(int n) { return 1024 / n < 1 ? 1 : (1024 / n > 16 ? 16 : 1024 / n); }
__host__ __device__ constexpr int fft_cols_per_item(int n) {
    return n == 512 ? 8 : (n > 256 ? 4 : (n == 256 || n == 192 ? 8 : 16));
}
// LDS of a column item without the measurement and mask strips (the raw passes)
__host__ __device__ constexpr int fft_cols_raw_lds(int n) { return (fft_cols_per_item(n) * n + n) * 8; }

struct ShearEntry {       // one (blade, bin): taps at rows y+oy(+1), columns x+ox(+1)
    int ox, oy;
    float w00, w01, w10, w11;  // (1-fy)(1-fx), (1-fy)fx, fy(1-fx), fy fx
    int pad0, pad1;
};

struct BladeDev {
    int knot;            // first knot of the blade's interval (0 for static plans)
    int has0, has1;      // which unweighted knot projections exist
    float w0, w1;        // their blend weights (1 - a, a)
    int ox_min, ox_max, oy_min, oy_max;  // shear offset extents over all bins
    int pad;
};

struct KnotEntry {       // a blade part that reads (projection) / feeds (adjoint) a knot
    int blade, part;
    float weight;
    int pad;
};

struct ProjGroup {       // up to 4 * GW parts of one knot projected together
    int knot, e0, ne;
    int ox_min, ox_max, oy_min, oy_max;
    int pad;
};

struct KnotInfo {        // union of the shear extents of the parts feeding a knot
    int ox_min, ox_max, oy_min, oy_max;
};

struct Task {            // one work item; field meaning depends on the kernel
    int slice, a, b, c;
};

struct SliceDesc {
    int n, S, T, B;
    int nparts;                  // parts per blade in the work buffer (1 or 2)
    int nstage;
    int radix[kMaxStages];
    int radix_code;              // radix of stage i in bits [3i, 3i+3)
    int n_col_items;            // column work items per blade (loss partials per blade)
    const float2* tw;            // twiddles exp(-2 pi i j / n), j < n
    const uint8_t* mask;
    const ShearEntry* shear;     // [B][S]
    const BladeDev* blade;       // [B]
    const int* knot_ptr;         // [T+1] CSR offsets into knot_ent
    const KnotEntry* knot_ent;
    const ShearEntry* knot_tap;  // [entries][S] shear taps times the entry's weight
    const ProjGroup* groups;
    const KnotInfo* knots;       // [T]
    const float2* y;             // measured k-space or nullptr
    float2* vol[2];              // current volume = vol[step & 1]
    float2* m;
    float2* v;
    float2* work;
    float2* grad;                // gradient output of the operator path, or the data
                                 // gradient a step stores for a separate update pass
    float* loss_part;            // [B][n_col_items]
    int* step;                   // device step counter; nullptr for operator calls
    int step_limit;              // work items of slices with *step >= step_limit exit
    int optimizer, schedule;
    unsigned sched_seed;         // VP_SCHED_RANDOM
    float data_w;                // weight of the data term (residual and loss partials)
    float lr, beta1, beta2, adam_eps;
    float ln_beta1, ln_beta2;    // log(beta) in FP64, rounded: bias corrections -expm1(t ln beta)
    float tv_w, l1_w, tv_eps;
};

// The blade images at the two ends of the blade-aligned DFT passes (k_rows in
// COL_RAW_FWD / COL_INVERSE with live_n != 0): the forward row pass builds each grid row
// from row y of the blade image (knots blended, centred, divided by the kernel
// transform) instead of reading it, and the inverse row pass writes the row's centre,
// divided the same way, into the blade image instead of the grid.
struct NuEdge {
    const float2* img_in;   // blade images [B][parts][m][m] (forward)
    float2* img_out;        // blade images, part 0 of [B][parts][m][m] (inverse)
    const BladeDev* blade;  // knot blend of dynamic blades (forward, parts == 2)
    const float* dea;       // [m] 1 / (kernel transform) at the centred index x - m/2
    int parts;
};

struct KArgs {
    const SliceDesc* descs;      // device array, or nullptr to use `one`
    SliceDesc one;
    const Task* tasks;
    int ntasks;
    int mode;
    int split_bin;
    int accumulate;
    float2* out0;
    float2* out1;
    float2* out2;
    const float2* in0;
    double* dpart;
    int epi;                     // optimiser epilogue of GATHER_STEP and the update pass (EPI_*)
    int stream;                  // with epi == EPI_ADAM_TV: take the EPI_STREAM variant
    int live_n;                  // COL_RAW_FWD / COL_INVERSE: 0, or the size m of a centred image
                                 // in the frame: only rows [0, m - m/2) and [n - m/2, n) are
                                 // nonzero on input (forward) or needed on output (inverse)
    NuEdge nue;                  // with live_n != 0: the row passes' blade-image ends
    // A fit step's first kernel (snap) copies the step counters of slices 0 .. nslices - 1
    // to their snapshot words; its last kernel (snap) reads the step from the snapshot and,
    // with advance, its block 0 advances the counters (step_snapshot, step_advance).
    int snap;
    int advance;
    int nslices;
};

// The allocation of a fit's step counter holds, kSnapWord ints after the counter, the
// copy of the counter that the step's last kernel reads.
constexpr int kSnapWord = 32;

// Column pass modes.
// COL_INVERSE (column and inverse row pass): in-place unscaled inverse DFT of the frames at
// a.out0 (frame = the task's blade index), read from a.in0. COL_RAW_FWD: the same for the
// forward DFT (column pass and forward row pass).
enum { COL_STEP = 0, COL_FORWARD = 1, COL_ADJOINT = 2, COL_INVERSE = 3, COL_RAW_FWD = 4 };
// Blade-aligned sampling by gridding: Kaiser-Bessel kernel of width kNuWidth on a grid
// oversampled by kNuSigma, tabulated at kNuTable + 1 points over [0, kNuWidth / 2].
constexpr int kNuSigma = 2;
constexpr float kNuWidth = 6.0f;
constexpr int kNuTable = 4096;
// Gather epilogues.
enum { GATHER_STORE = 0, GATHER_STEP = 1 };
// Optimiser epilogue variants: EPI_GENERIC takes the optimiser and the regulariser
// weights from each slice's descriptor at run time; EPI_ADAM_TV is the same arithmetic
// compiled for slices that all run Adam with TV on and L1 off. EPI_STREAM (with
// EPI_ADAM_TV) makes the update's moment loads, its stores and its loads of the previous
// knot's planes non-temporal, for steps whose state exceeds kStreamState; it changes no
// result.
enum { EPI_GENERIC = 0, EPI_ADAM_TV = 1, EPI_STREAM = 2 };
__host__ __device__ constexpr bool epi_fast(int e) { return (e & EPI_ADAM_TV) != 0; }
// cache-policy operand of the update's streamed loads and stores (2: non-temporal)
__host__ __device__ constexpr int epi_cache(int e) { return (e & EPI_STREAM) ? 2 : 0; }
// A step whose optimiser state (both volume copies and the Adam moments) exceeds the
// 256 MiB Infinity Cache streams it (EPI_STREAM): the state cannot stay cached from one
// step to the next, and keeping the data read or written for the last time out of the
// caches leaves them to the volume planes that neighbouring work items read again. A smaller state
// stays cached between steps and is not streamed.
constexpr size_t kStreamState = (size_t)256 << 20;
__host__ __device__ constexpr int epi_for(int optimizer, float tv_w, float l1_w) {
    return (optimizer == VP_OPT_ADAM && tv_w != 0.f && l1_w == 0.f) ? EPI_ADAM_TV : EPI_GENERIC;
}

}  // namespace vp
