/*
 * vp.h -- C ABI of the MI355X lifted-PROPELLER reconstruction library (libvp.so).
 *
 * The library fits a complex (x, y, spectral-offset[, time]) voxel grid to
 * PROPELLER blade measurements (Ghosh, Wetzstein, Pilanci, Fridovich-Keil,
 * CVPR 2024). Its operations follow the paper's statement of the problem:
 *
 *   volume V[t][s][y][x]    complex, Section 4.1 (static grid; a dense grid of T
 *                           time knots for dynamic scans, or the paper's complex
 *                           K-Planes model through the vp_kplanes_* calls)
 *   forward  A V            Section 4.2: for every blade b, sum over spectral bins
 *                           s of the bin's image shifted by delta_s along the
 *                           blade's readout direction (bilinear, zero outside the
 *                           grid), unitary 2D DFT, blade k-space mask (or the
 *                           blade-aligned samples of Section 7's non-uniform DFT,
 *                           vp_nu_* calls)
 *   objective               Section 4.3: 0.5 sum_b |M_b(A V)_b - M_b y_b|^2
 *                           + tv_weight TV(V) + l1_weight L1(V)
 *   optimiser               Section 4.3: Adam (or plain gradient descent)
 *   outputs                 Section 4.3 render at phi = 0 (sum over s), and the
 *                           fat/water split of Section 6 (bins below split_bin are
 *                           water, the rest fat)
 *
 * Conventions for every call:
 *   - Every call returns vp_status: VP_OK (0) or a negative error code. No C++
 *     exception crosses this boundary. vp_last_error() gives a thread-local
 *     message for the last failing call on the calling thread.
 *   - Complex arrays are interleaved (re, im) float32 pairs, C order, x fastest:
 *     volumes [T][S][n][n], blade arrays [B][n][n], renders [T][n][n].
 *   - k-space arrays use unshifted DFT order: index j holds the signed frequency
 *     j for j <= (n-1)/2 and j - n otherwise, on both axes; the DFT is unitary.
 *   - Angles are radians; shifts are pixels; blade times lie in [0, 1].
 *   - The caller owns every buffer it passes. Opaque handles are released by
 *     their *_destroy call, which accepts NULL.
 *   - Plans are immutable after creation and may be shared between threads.
 *   - "d_" pointers are device pointers on the current HIP device (for example
 *     torch tensor storage): contiguous, 8-byte aligned, not aliased with each
 *     other. Calls that take a `stream` (a hipStream_t, NULL = the null stream)
 *     are asynchronous on it. All other pointers are host pointers.
 *   - Device memory exhaustion yields VP_ERR_NOMEM; a failing HIP runtime call
 *     yields VP_ERR_DEVICE.
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vp_status;

enum {
    VP_OK = 0,
    VP_ERR_ARG = -1,          /* NULL, non-finite or out-of-range argument */
    VP_ERR_UNSUPPORTED = -2,  /* valid problem this build does not handle (size, shift range) */
    VP_ERR_DEVICE = -3,       /* HIP runtime failure or no usable device */
    VP_ERR_NONFINITE = -4,    /* non-finite measurement, or the objective became non-finite */
    VP_ERR_BUDGET = -5,       /* a server request larger than the whole memory budget */
    VP_ERR_NOMEM = -6,        /* device or host allocation failed */
    VP_ERR_TIMEOUT = -7,      /* vp_server_wait timed out; the request keeps running */
    VP_ERR_CANCELLED = -8,    /* the request was cancelled before it finished */
    VP_ERR_NOT_FOUND = -9,    /* unknown request id */
    VP_ERR_STATE = -10        /* call not valid in the object's current state */
};

typedef struct { float re, im; } vp_c64;

typedef struct vp_plan vp_plan;
typedef struct vp_session vp_session;
typedef struct vp_server vp_server;
typedef struct vp_kplanes_session vp_kplanes_session;
typedef struct vp_nu_session vp_nu_session;

/* Acquisition geometry (Section 4.2 "Projection" and "Blur").
 *   n              image side; the grid is n x n and each blade's readout has n
 *                  samples. Supported: 1 <= n <= 512 with no prime factor above 5.
 *   n_spec         spectral bins S >= 1 (at most 256).
 *   n_time         time knots T >= 1 (at most 64); 1 = static. Knot k sits at
 *                  time k/(T-1); a blade at time tau sees the linear blend of
 *                  knots floor(tau (T-1)) (clamped to T-2) and the next one.
 *   n_blades       B >= 1 (at most 256).
 *   angle_rad[B]   blade readout direction u_b = (cos, sin) in (x = column,
 *                  y = row); finite.
 *   lines[B]       blade width in k-space lines, 1 <= L <= n. The blade's
 *                  support is the half-open rotated rectangle of length n along
 *                  u_b and width L across it, ties broken by a 1e-9 margin.
 *   blade_time[B]  acquisition time of each blade in [0, 1]; must be NULL iff
 *                  n_time == 1.
 *   spec_shift_px[S]  displacement, in pixels along u_b, of spectral bin s
 *                  (tan(phi) times its off-resonance); finite, |shift| <= 16. */
typedef struct {
    int32_t n;
    int32_t n_spec;
    int32_t n_time;
    int32_t n_blades;
    const double* angle_rad;
    const int32_t* lines;
    const double* blade_time;
    const double* spec_shift_px;
} vp_geometry;

enum { VP_OPT_ADAM = 0, VP_OPT_GD = 1 };
enum { VP_SCHED_ALL_BLADES = 0, VP_SCHED_CYCLIC = 1, VP_SCHED_RANDOM = 2 };

/* Fit settings (Section 4.3). tv_eps is the Charbonnier epsilon of both the TV
 * and the L1 term. A step is one optimiser update on the gradient summed over
 * all blades (VP_SCHED_ALL_BLADES) or over one blade, the paper's one-blade-per-
 * iteration schedule: blade (t-1) mod B (VP_SCHED_CYCLIC) or a blade drawn at
 * random, splitmix64(seed * 2^32 + t - 1) mod B with SplitMix64 of Steele, Lea and
 * Flood (VP_SCHED_RANDOM). data_weight multiplies the data term: the image-space
 * and k-space squared errors of Section 4.3 are the same number under the unitary
 * DFT, so their weights add up to this one factor (default 1, must be > 0). The
 * volume starts at zero unless an initial volume is given. split_bin < 0 means S/2. */
/* Tile shape of the projection, gather and update kernels: how the work is cut
 * into work items, never what is computed (every shape gives the same results bit
 * for bit). proj_rows: rows of a projection tile, in {1, 2, 4, 8, 12}; proj_parts:
 * blade parts per wave of a projection item, in {1, 2, 4, 8}, with proj_rows *
 * proj_parts <= 16 (12 rows: one part); gath_rows: rows of a gather tile, in {2, 4}; gath_bins:
 * spectral bins per wave of a gather item, in {1, 2, 4, 8}, with gath_rows *
 * gath_bins <= 16 unless gath_resident is 1; upd_bins: 0 runs the regulariser and optimiser update inside
 * the gather kernel, 2, 4 or 8 runs it as a separate pass (that many bins per
 * wave) over a stored data gradient (one more volume-sized device buffer);
 * gath_waves: waves per gather item, 4 or 8 (0 means 4), which share the item's
 * staged blade regions, so an item covers gath_waves * gath_bins bins; proj_waves:
 * waves per projection item, 4 or 8 (0 means 4), which share the item's staged
 * volume regions, so an item projects proj_waves * proj_parts blade parts;
 * gath_resident: 1 stages every blade part feeding a knot at once and interleaves
 * each bin's gather with that bin's update (needs upd_bins 0, at most 32 parts per
 * knot, staged regions of at most 2048 elements and 64 KiB of LDS per item;
 * VP_ERR_UNSUPPORTED otherwise), 0 stages the parts a few at a time. A tile is 64
 * columns wide. All fields 0: the plan's own (or autotuned) shape. */
typedef struct {
    int32_t proj_rows;
    int32_t proj_parts;
    int32_t gath_rows;
    int32_t gath_bins;
    int32_t upd_bins;
    int32_t gath_waves;
    int32_t proj_waves;
    int32_t gath_resident;
} vp_tiles;

typedef struct {
    float tv_weight;
    float l1_weight;
    float tv_eps;
    int32_t n_steps;
    int32_t optimizer;
    float lr;
    float beta1;
    float beta2;
    float adam_eps;
    int32_t schedule;
    int32_t split_bin;
    int32_t device;
    /* Tile shape. All fields 0: the shape recorded by vp_plan_tune for a plan of
     * the same sizes on this device if there is one, else (autotune != 0) tune now
     * and record it, else the plan's built-in choice. Otherwise the shape given,
     * which must be valid for the plan (VP_ERR_UNSUPPORTED if not). */
    vp_tiles tiles;
    int32_t autotune;
    uint32_t seed;       /* VP_SCHED_RANDOM */
    float data_weight;   /* > 0 */
} vp_options;

/* Fills defaults: tv_weight 1e-3, l1_weight 0, tv_eps 1e-3, n_steps 200, Adam
 * with lr 1e-2, betas (0.9, 0.999), eps 1e-8, all-blades schedule, split S/2,
 * device 0, automatic tile shape without tuning, seed 0, data_weight 1. */
vp_status vp_options_default(vp_options* opts);

/* Static description of a status code; never NULL. */
const char* vp_status_string(vp_status status);

/* Thread-local message for the last failing call on this thread ("" if none). */
const char* vp_last_error(void);

/* ------------------------------------------------------------------ plans */

/* Validates the geometry and builds the host-side plan: blade masks (evaluated
 * in FP64), the per-(blade, bin) bilinear shear table, blade-to-knot weights,
 * DFT twiddles and launch tables. Touches no device. Errors: VP_ERR_ARG for
 * NULL or non-finite input, sizes below 1, lines outside [1, n], blade times
 * outside [0, 1] or a blade_time pointer that disagrees with n_time;
 * VP_ERR_UNSUPPORTED for n, S, T or B above the limits above, n with a prime
 * factor above 5, or shifts beyond 16 px. *out is set only on success. */
vp_status vp_plan_create(const vp_geometry* geometry, vp_plan** out);

/* Releases the plan and any per-device tables it holds. NULL is a no-op. The
 * plan must not be in use by a running call, session or server request. */
vp_status vp_plan_destroy(vp_plan* plan);

/* Sizes of a plan. Any output pointer may be NULL. */
vp_status vp_plan_shape(const vp_plan* plan, int32_t* n, int32_t* n_spec, int32_t* n_time, int32_t* n_blades);

/* Blade b's k-space support as n*n bytes (1 = measured), unshifted order. */
vp_status vp_plan_mask(const vp_plan* plan, int32_t b, uint8_t* out_n_by_n);

/* Shear of blade b, bin s: the blade image at (x, y) takes bilinear taps of bin
 * s at rows y+oy, y+oy+1 and columns x+ox, x+ox+1 with fractional weights
 * (fx, fy), where (ox, oy) = floor(-d) and (fx, fy) = -d - floor(-d) for the
 * displacement d = spec_shift_px[s] * u_b. Any output pointer may be NULL. */
vp_status vp_plan_shear(const vp_plan* plan, int32_t b, int32_t s, int32_t* ox, int32_t* oy, float* fx, float* fy);

/* Knot index k and blend weight a of blade b (0 and 0 for static plans). */
vp_status vp_plan_knot(const vp_plan* plan, int32_t b, int32_t* knot, float* alpha);

/* Exact device bytes one reconstruction of this plan allocates with these
 * options (volume ping-pong, Adam moments, blade work images, measurements,
 * tables, partial sums). Used for admission by memory budget. */
vp_status vp_plan_device_bytes(const vp_plan* plan, const vp_options* opts, uint64_t* bytes);

/* Autotuner: times every compiled tile shape that fits the plan on opts->device
 * (projection launches per projection shape; the fused gather/update per gather
 * shape; the gather that stores the data gradient per gather shape and the
 * separate update pass per update shape; a few repetitions each, on a scratch
 * reconstruction state with zero measurements; the optimiser and regulariser
 * settings of opts select the update that is timed),
 * records the fastest shape for plans of the same sizes, shear extents and
 * optimiser in a process-wide table and returns it. Sessions, reconstructions,
 * batches and operators created later pick it up (vp_options.tiles all zero).
 * Allocates about vp_plan_device_bytes on the device for the duration of the call.
 * Errors: VP_ERR_ARG for NULL arguments or bad options, VP_ERR_NOMEM,
 * VP_ERR_DEVICE. */
vp_status vp_plan_tune(const vp_plan* plan, const vp_options* opts, vp_tiles* out);

/* The tile shape a session created with `opts` would use now (no measuring unless
 * opts->autotune asks for it and no shape is recorded yet). */
vp_status vp_plan_tiles(const vp_plan* plan, const vp_options* opts, vp_tiles* out);

/* ------------------------------------------------------------------ operators (device pointers) */

/* d_out[B][n][n] = M_b . DFT2(P_b V) - (d_y ? M_b . d_y : 0): the forward model
 * of Section 4.2 applied to d_vol[T][S][n][n]. Device scratch of B*n*n complex
 * values (twice that when T > 1) is taken from the stream-ordered allocator
 * and released on the stream. */
vp_status vp_forward(const vp_plan* plan, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out, void* stream);

/* vp_forward without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same kernels and results as vp_forward, bit for bit, with the blade work images in a
 * fixed 32 MiB device array that the library keeps on each device it runs on until the
 * process ends. It calls no allocator: the plan's device tables must already be on the
 * current device (any earlier vp_forward, vp_adjoint, session or reconstruction of the
 * plan there uploads them). Every call on one device shares that device's array, so
 * calls that overlap on one device (concurrent streams or threads) race; calls ordered
 * on one stream do not. Errors: VP_ERR_ARG for NULL pointers; VP_ERR_UNSUPPORTED when
 * the plan needs more than 32 MiB of blade images (B * n * n complex values, twice that
 * when T > 1); VP_ERR_STATE when the plan's tables are not on the current device. */
vp_status vp_forward_noalloc(const vp_plan* plan, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out,
                             void* stream);

/* d_grad[T][S][n][n] (+)= A^H d_kres: blade mask, unitary inverse DFT and the
 * transpose of the sheared projection (a gather, no atomics), with dynamic
 * blades split onto their two knots with weights (1-a, a). For a real loss
 * L(A V) with dL/d(AV) = d_kres (as dL/dRe + i dL/dIm) this is dL/dRe V +
 * i dL/dIm V. accumulate != 0 adds to d_grad, otherwise overwrites it. */
vp_status vp_adjoint(const vp_plan* plan, const vp_c64* d_kres, vp_c64* d_grad, int32_t accumulate, void* stream);

/* Blade-aligned sampling (the non-uniform DFT that the paper's discussion names for
 * real PROPELLER data, in place of the Cartesian mask and DFT). Blade b's samples sit
 * on its rotated lattice k = r u_b + q n_b, r = j - n/2 (j < n), q = l - L_b/2
 * (l < L_b), u_b = (cos, sin), n_b = (-sin, cos); sample arrays are [B][Lmax][n]
 * (Lmax = the largest L_b, lines l >= L_b unused: written as 0, read as ignored).
 * Forward: d_out = (1/n) sum_x P_b(x) exp(-2 pi i k.x / n) - d_y (d_y may be NULL), by
 * gridding (Kaiser-Bessel kernel of width 6 on a grid oversampled 2x; about 1e-5 of the
 * definition). Adjoint: d_grad (+)= the exact transpose of the forward (gather form, no
 * atomics). Device pointers on the plan's device, asynchronous on `stream`; scratch of
 * B (2n)^2 complex values plus the blade images comes from the stream-ordered
 * allocator. VP_ERR_UNSUPPORTED if 2n is above the largest transform length (512). */
vp_status vp_nu_forward(const vp_plan* plan, const vp_c64* d_vol, const vp_c64* d_y, vp_c64* d_out, void* stream);
vp_status vp_nu_adjoint(const vp_plan* plan, const vp_c64* d_samples, vp_c64* d_grad, int32_t accumulate,
                        void* stream);

/* The fit of Section 4.3 on blade-aligned samples, as a resident session: the Cartesian
 * session's projection, fused gather and update, regularisers, schedules (all blades or
 * one per step, as in vp_reconstruct) and step counter, with the gridding passes above in
 * place of the masked Cartesian DFT. samples: host [B][Lmax][n] (the layout above; lines
 * l >= L_b ignored); init as in vp_session_create. VP_ERR_NONFINITE if a used sample is
 * NaN or Inf; VP_ERR_UNSUPPORTED if 2n is above 512. Device memory: the Cartesian session's plus B (2n)^2 complex values and two
 * sample arrays, freed by vp_nu_session_destroy. */
vp_status vp_nu_session_create(const vp_plan* plan, const vp_options* opts, const vp_c64* samples,
                               const vp_c64* init, vp_nu_session** out);

/* n_steps optimiser steps (use_graph != 0: one captured step replayed), then waits. */
vp_status vp_nu_session_step(vp_nu_session* session, int32_t n_steps, int32_t use_graph);

/* Profiling: n_steps more steps eagerly with a HIP event around every stage; mean
 * milliseconds to stage_ms[8]: projection, forward row DFT of the grids (built from the
 * blade images), forward column DFT, interpolation (residual and loss partials), spread,
 * inverse column DFT, inverse row DFT (written back into the blade images), and the
 * gather with the regulariser gradient, update and step counter. */
vp_status vp_nu_session_stage_times(vp_nu_session* session, int32_t n_steps, double* stage_ms);

/* Current volume and renders to host buffers (any may be NULL) and, if objective is
 * not NULL, 0.5 data_weight sum |r|^2 + TV + L1 at the current volume. */
vp_status vp_nu_session_read(vp_nu_session* session, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out,
                             vp_c64* fat_out, double* objective);

/* Checkpoint and resume, as vp_session_get_state / vp_session_set_state: the volume,
 * the Adam moments and the step count (a resumed fit continues bit for bit). */
vp_status vp_nu_session_get_state(vp_nu_session* session, vp_c64* volume, vp_c64* m, vp_c64* v, int64_t* step);
vp_status vp_nu_session_set_state(vp_nu_session* session, const vp_c64* volume, const vp_c64* m, const vp_c64* v,
                                  int64_t step);

vp_status vp_nu_session_destroy(vp_nu_session* session);

/* One synchronous fit on blade-aligned samples: create, opts->n_steps steps, read
 * (final_loss is the objective there), destroy. */
vp_status vp_nu_reconstruct(const vp_plan* plan, const vp_options* opts, const vp_c64* samples, const vp_c64* init,
                            vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out,
                            double* final_loss);

/* d_grad (+)= tv_weight * grad TV(d_vol) + l1_weight * grad L1(d_vol)
 * (Section 4.3: Charbonnier TV over x, y, s and t with forward differences
 * where the neighbour exists; Charbonnier L1). */
vp_status vp_tv_grad(const vp_plan* plan, const vp_c64* d_vol, float tv_weight, float l1_weight, float tv_eps,
                     vp_c64* d_grad, int32_t accumulate, void* stream);

/* One optimiser step of Section 4.3 on caller-held state: g = d_grad (the data-term
 * gradient as dL/dRe + i dL/dIm, e.g. from vp_adjoint, weighted by the caller) +
 * tv_weight grad TV(d_vol) + l1_weight grad L1(d_vol) (weights and eps from opts), then
 * opts' optimiser: Adam with the bias corrections of step t >= 1 and the moments d_m,
 * d_v (each [T][S][n][n] of (re, im) pairs, updated in place; NULL allowed for GD) or GD.
 * The new volume goes to d_vol_out, which must not overlap d_vol (the TV stencil reads
 * the old one). The same per-voxel arithmetic as the update of vp_reconstruct. Device
 * pointers on the plan's device, asynchronous on `stream`. */
vp_status vp_step(const vp_plan* plan, const vp_options* opts, const vp_c64* d_vol, const vp_c64* d_grad,
                  vp_c64* d_m, vp_c64* d_v, int64_t t, vp_c64* d_vol_out, void* stream);

/* Section 4.3 render at phi = 0 and the Section 6 split: d_proj[t] = sum over
 * all bins, d_water = bins [0, split), d_fat = bins [split, S); split_bin < 0
 * means S/2. Any output may be NULL. */
vp_status vp_render(const vp_plan* plan, const vp_c64* d_vol, int32_t split_bin, vp_c64* d_proj, vp_c64* d_water,
                    vp_c64* d_fat, void* stream);

/* ------------------------------------------------------------------ evaluation (device pointers) */

/* Baseline reconstructions of Section 6 (evaluation): frame f is the unitary
 * inverse DFT of the coverage-weighted k-space average of the blades
 * max(0, f - window + 1) .. f, i.e. at each sample the mean of the values of those
 * blades whose mask holds it (zero where none does). window <= 0 takes every blade
 * up to f, so window = B (or 0) and f = B - 1 is the static baseline that combines
 * all blades, and window = 5 the dynamic one over the five most recent blades.
 * d_kspace: device [B][n][n] measurements (off-mask values are ignored).
 * d_out: device [n_frames][n][n], frames first_frame .. first_frame + n_frames - 1,
 * image space; it must not overlap d_kspace. Asynchronous on `stream`; allocates
 * nothing. Errors: VP_ERR_ARG for NULL pointers (with n_frames > 0), first_frame < 0,
 * n_frames < 0, first_frame + n_frames > B, or overlapping buffers. */
vp_status vp_baseline(const vp_plan* plan, const vp_c64* d_kspace, int32_t window, int32_t first_frame,
                      int32_t n_frames, vp_c64* d_out, void* stream);

/* PSNR on magnitudes (Section 6, quantitative results): for each of n_images
 * consecutive images of n_px complex samples in d_image and d_truth (device),
 * d_terms[3 i + 0] = mean over samples of (|image| - |truth|)^2 (FP64),
 * d_terms[3 i + 1] = peak = max |truth|, d_terms[3 i + 2] = 10 log10(peak^2 / mse)
 * (+inf when mse = 0). Deterministic; runs on the current device, asynchronous on
 * `stream`; allocates nothing. Errors: VP_ERR_ARG for NULL pointers (with
 * n_images > 0), n_px < 1 or n_images < 0. */
vp_status vp_psnr(const vp_c64* d_image, const vp_c64* d_truth, int64_t n_px, int32_t n_images, double* d_terms,
                  void* stream);

/* ------------------------------------------------------------------ sessions (resident state) */

/* Uploads kspace[B][n][n] (host; off-mask values are ignored) and the initial
 * volume (host [T][S][n][n], NULL = zeros) to opts->device and allocates the
 * optimiser state there. VP_ERR_NONFINITE if kspace holds NaN or Inf. */
vp_status vp_session_create(const vp_plan* plan, const vp_options* opts, const vp_c64* kspace, const vp_c64* init,
                            vp_session** out);

/* Runs n_steps optimiser steps on the device (use_graph != 0: one captured
 * step replayed) and waits for them. */
vp_status vp_session_step(vp_session* session, int32_t n_steps, int32_t use_graph);

/* Steps taken so far. */
vp_status vp_session_steps_done(const vp_session* session, int64_t* steps);

/* Copies the current volume and renders to host buffers; any may be NULL. */
vp_status vp_session_read(vp_session* session, vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out,
                          vp_c64* fat_out);

/* Objective (data + weighted TV and L1) at the current volume, over all blades. */
vp_status vp_session_objective(vp_session* session, double* objective, double* data_term);

/* Checkpoint: copies volume, Adam moments (interleaved (re, im) pairs, each
 * shaped like the volume) and the step count to host buffers. */
vp_status vp_session_get_state(vp_session* session, vp_c64* volume, vp_c64* m, vp_c64* v, int64_t* step);

/* Resume: restores what vp_session_get_state returned. */
vp_status vp_session_set_state(vp_session* session, const vp_c64* volume, const vp_c64* m, const vp_c64* v,
                               int64_t step);

/* Profiling: runs n_steps more steps eagerly on the session stream with a HIP
 * event recorded before and after every stage, and writes the mean duration in
 * milliseconds of each stage to stage_ms[5]: projection, forward row DFT,
 * column pass (DFT, mask, residual, inverse DFT), inverse row DFT, and the
 * gather with the regulariser gradient and optimiser update (whose first block
 * also advances the step counter). */
vp_status vp_session_stage_times(vp_session* session, int32_t n_steps, double* stage_ms);

vp_status vp_session_destroy(vp_session* session);

/* ------------------------------------------------------------------ whole reconstructions */

/* One synchronous reconstruction: opts->n_steps steps from init (NULL = zero)
 * on opts->device. Outputs (host, any may be NULL): volume [T][S][n][n], proj,
 * water, fat [T][n][n], and the objective at the returned volume. */
vp_status vp_reconstruct(const vp_plan* plan, const vp_options* opts, const vp_c64* kspace, const vp_c64* init,
                         vp_c64* volume_out, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out,
                         double* final_loss);

/* Output slots of one batched or served reconstruction; NULL pointers skip. */
typedef struct {
    vp_c64* volume_out;
    vp_c64* proj_out;
    vp_c64* water_out;
    vp_c64* fat_out;
    double final_loss;
    int64_t steps_done;
    vp_status status;
} vp_result;

/* Many independent slices, possibly of different sizes, reconstructed together
 * on opts[0]->device: each step is one launch per stage over the concatenated work
 * items of all slices (a block per work item, each reading its slice's descriptor
 * from a device table; the hardware dispatcher balances the uneven items), the whole
 * step captured once in a HIP graph and replayed. Every slice's result is
 * the one vp_reconstruct gives it alone (bit for bit: summation orders do not
 * depend on the batch). Per-slice status goes to results[i]->status; the call
 * returns the first failure, if any. */
vp_status vp_batch_reconstruct(int32_t n, const vp_plan* const* plans, const vp_options* const* opts,
                               const vp_c64* const* kspace, vp_result* const* results);

/* A resident batch: the slices of vp_batch_reconstruct uploaded once and stepped
 * together, for callers that step, time or read a batch in parts. vp_batch_create
 * uploads every slice (kspace[i] host [B_i][n_i][n_i]) to opts[0]->device, picks the
 * batch's tile shape as vp_batch_reconstruct does and builds the concatenated work
 * lists; a slice that cannot be set up is reported by vp_batch_read (the call returns
 * its status, the others still run). *out stays NULL if no slice could be set up.
 * vp_batch_step runs n_steps batched steps (use_graph != 0: one captured step replayed;
 * slice i stops at opts[i]->n_steps) and waits. vp_batch_stage_times runs n_steps more
 * eagerly with a HIP event around each stage (stage_ms[5] as in vp_session_stage_times,
 * each stage one launch over all slices). vp_batch_read copies slice i's outputs and its
 * objective into *result (NULL output pointers skip). */
typedef struct vp_batch vp_batch;
vp_status vp_batch_create(int32_t n, const vp_plan* const* plans, const vp_options* const* opts,
                          const vp_c64* const* kspace, vp_batch** out);
vp_status vp_batch_step(vp_batch* batch, int32_t n_steps, int32_t use_graph);
vp_status vp_batch_stage_times(vp_batch* batch, int32_t n_steps, double* stage_ms);
vp_status vp_batch_read(vp_batch* batch, int32_t i, vp_result* result);
vp_status vp_batch_destroy(vp_batch* batch);

/* ------------------------------------------------------------------ K-Planes dynamic model */

/* The complex K-Planes volume model of Section 4.1 (its equation and the paragraph
 * after it). For each scale c, six complex grids of F features,
 *   xy [R_c][R_c][F] (row y), x-omega [S][R_c][F], y-omega [S][R_c][F],
 *   xt [R_t][R_c][F], yt [R_t][R_c][F], omega-t [R_t][S][F],
 * stored in this order, scale after scale, in one flat complex vector followed by the
 * weight vector a [F]. The value at voxel (x, y, s) and time tau is
 *   sum_c sum_f a_f * prod over the six grids of feature f read there,
 * each grid read by linear interpolation along its axes: index i of an axis of m
 * samples sits at i (R - 1) / (m - 1) on an axis of R nodes, tau at tau (R_t - 1); bins
 * are read at the S nodes of the omega axis. A fit step evaluates the model at every
 * blade's time (the plan's blade times, 0 for a static plan), projects and blurs it as
 * in Section 4.2 and minimises the data term of Section 4.3 plus the grid regularisers
 * below by Adam or GD on (Re, Im) of every parameter. */
#define VP_KP_MAX_SCALES 2
typedef struct {
    int32_t features;                       /* F: 1, 2, 4, 8 or 16 */
    int32_t time_res;                       /* R_t >= 1 */
    int32_t n_scales;                       /* 1 .. VP_KP_MAX_SCALES */
    int32_t spatial_res[VP_KP_MAX_SCALES];  /* R_c in [1, n] */
    float tv_weight;                        /* Charbonnier TV along the grids' x, y and omega axes */
    float smooth_weight;                    /* squared second differences along t of the time grids */
    float sparse_weight;                    /* Charbonnier modulus of (p - 1) on the time grids */
    float eps;                              /* Charbonnier epsilon, > 0 */
} vp_kplanes;

/* Number of complex parameters of the model for the plan's n and S. Host only.
 * Errors: VP_ERR_ARG for NULL arguments or an invalid model (sizes out of range,
 * non-finite weights, eps <= 0). */
vp_status vp_kplanes_param_count(const vp_plan* plan, const vp_kplanes* model, int64_t* count);

/* d_vol[n_times][S][n][n] = the model d_params at the host times[n_times] (each in
 * [0, 1]). Device pointers on the current device; runs on `stream` and returns when it
 * has finished (it stages small tables through host memory). */
vp_status vp_kplanes_decode(const vp_plan* plan, const vp_kplanes* model, const vp_c64* d_params,
                            const double* times, int32_t n_times, vp_c64* d_vol, void* stream);

/* d_grad = gradient (dL/dRe + i dL/dIm) with respect to d_params of
 * L = 0.5 sum_b |M_b DFT2(P_b f(., tau_b)) - M_b y_b|^2 + the grid regularisers, for
 * device k-space d_kspace[B][n][n]; *objective = L and *data_term = the first sum (either
 * may be NULL). Runs on `stream` and returns when it has finished. Device scratch (two
 * dense [B][S][n][n] volumes and the factors) comes from the stream-ordered allocator. */
vp_status vp_kplanes_gradient(const vp_plan* plan, const vp_kplanes* model, const vp_c64* d_params,
                              const vp_c64* d_kspace, vp_c64* d_grad, double* objective, double* data_term,
                              void* stream);

/* Resident fit: uploads kspace[B][n][n] and the initial parameters init[count] (host)
 * to opts->device. opts gives n_steps (unused here), optimizer, lr, beta1, beta2,
 * adam_eps, data_weight, device and autotune (the blade kernels of the fit take the
 * tile shape recorded for the geometry with one knot per blade, tuned first when
 * autotune is set and none is recorded); tv_weight / l1_weight are ignored (the model
 * carries its own weights); only VP_SCHED_ALL_BLADES is supported
 * (VP_ERR_UNSUPPORTED otherwise). */
vp_status vp_kplanes_session_create(const vp_plan* plan, const vp_kplanes* model, const vp_options* opts,
                                    const vp_c64* kspace, const vp_c64* init, vp_kplanes_session** out);

/* n_steps optimiser steps (use_graph != 0: one captured step replayed); waits. */
vp_status vp_kplanes_session_step(vp_kplanes_session* session, int32_t n_steps, int32_t use_graph);

/* Copies the parameters (params_out[count], may be NULL) and renders the model at the
 * host frame_times[n_frames]: proj_out = sum over bins, water_out = bins below
 * opts->split_bin (S/2 if negative), fat_out = the rest, each [n_frames][n][n] and may
 * be NULL; *objective (may be NULL) = L at the current parameters. */
vp_status vp_kplanes_session_read(vp_kplanes_session* session, vp_c64* params_out, int32_t n_frames,
                                  const double* frame_times, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out,
                                  double* objective);

/* Profiling: n_steps more eager steps with HIP events around each stage; stage_ms[6] =
 * mean milliseconds of: factors and dense decode; projection, DFT passes and adjoint
 * gather; the gradient of the xy factor; of the x factor; of the y factor; grid
 * gradients, regularisers and update. */
vp_status vp_kplanes_session_stage_times(vp_kplanes_session* session, int32_t n_steps, double* stage_ms);

/* Checkpoint and resume: the parameter vector, its Adam moments (each [count] complex,
 * (re, im) pairs) and the step count, to and from host buffers; set_state with NULL
 * moments starts them at zero. A resumed fit continues bit for bit. */
vp_status vp_kplanes_session_get_state(vp_kplanes_session* session, vp_c64* params, vp_c64* m, vp_c64* v,
                                       int64_t* step);
vp_status vp_kplanes_session_set_state(vp_kplanes_session* session, const vp_c64* params, const vp_c64* m,
                                       const vp_c64* v, int64_t step);

vp_status vp_kplanes_session_destroy(vp_kplanes_session* session);

/* Whole fit: session_create, opts->n_steps graph-replayed steps, session_read, destroy. */
vp_status vp_kplanes_reconstruct(const vp_plan* plan, const vp_kplanes* model, const vp_options* opts,
                                 const vp_c64* kspace, const vp_c64* init, vp_c64* params_out, int32_t n_frames,
                                 const double* frame_times, vp_c64* proj_out, vp_c64* water_out, vp_c64* fat_out,
                                 double* final_loss);

/* ------------------------------------------------------------------ serving */

/* A reconstruction server on one device: requests are admitted in arrival order
 * while the sum of their vp_plan_device_bytes stays within hbm_budget and at most
 * max_slots are resident; an admitted request keeps its state on the device until it
 * finishes. The oldest resident requests with work left (up to four, and only until
 * their volumes reach 8M voxels, at least one) each replay their own captured step on
 * their own stream, eight steps per enqueued super-step with up to two super-steps in
 * flight each, so their work overlaps on the device; requests that arrive meanwhile
 * are admitted (their state uploaded) as slots and memory free up and start stepping
 * as soon as an older one finishes (continuous batching). A request's result does not
 * depend on the mix it ran in. The server is thread-safe. */
vp_status vp_server_create(int32_t device, uint64_t hbm_budget, int32_t max_slots, vp_server** out);

/* Queues a request. The inputs are copied before the call returns (plan is
 * referenced and must outlive the request). VP_ERR_BUDGET if the request alone
 * exceeds the budget; VP_ERR_NONFINITE for a non-finite kspace. */
vp_status vp_server_submit(vp_server* server, const vp_plan* plan, const vp_options* opts, const vp_c64* kspace,
                           uint64_t* request_id);

/* Waits up to timeout_us (< 0: forever) for a request, then copies its outputs
 * into *result and forgets it. Returns the request's status, VP_ERR_TIMEOUT,
 * or VP_ERR_NOT_FOUND. */
vp_status vp_server_wait(vp_server* server, uint64_t request_id, int64_t timeout_us, vp_result* result);

/* Non-blocking: *done = 1 when the request has finished (or failed). */
vp_status vp_server_poll(vp_server* server, uint64_t request_id, int32_t* done);

/* Cancels a queued or running request; its wait returns VP_ERR_CANCELLED. */
vp_status vp_server_cancel(vp_server* server, uint64_t request_id);

/* Latency statistics in microseconds (completion minus submission) over
 * finished requests, and completed requests per second of server wall time. */
vp_status vp_server_stats(vp_server* server, double* p50_us, double* p99_us, double* throughput_rps,
                          int64_t* completed);

/* Stops the worker after the running super-step; unfinished requests fail
 * with VP_ERR_CANCELLED. */
vp_status vp_server_destroy(vp_server* server);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */
