// Complex K-Planes dynamic volume model (Section 4.1): device descriptor and launchers.
//
// Parameters (complex, one flat vector): for each scale c the grids xy [R_c][R_c][F]
// (row y), x-omega [S][R_c][F], y-omega [S][R_c][F], xt [R_t][R_c][F], yt [R_t][R_c][F],
// omega-t [R_t][S][F], then the weight vector a [F]. The value at voxel (x, y, s) and
// time tau is sum_c sum_f a_f * prod over the six grids of feature f, each read by linear
// interpolation along its axes.
//
// A fit step evaluates the model at every blade's time with the separable factors
//   XA_c[b][s][x][f] = a_f * Xs_c[s][x][f] * qx_c[b][x][f] * qs_c[b][s][f]
//   Yf_c[b][s][y][f] = Ys_c[s][y][f] * qy_c[b][y][f]
//   Z_c[y][x][f]     = xy_c read at (y, x)
// (Xs, Ys: the x-omega and y-omega grids read at x or y; qx, qy, qs: the time grids read
// at the blade's time and at x, y or s), so V_b[s][y][x] = sum_c sum_f Z XA Yf. The dense
// per-blade volumes go through the lifted projection, blur and adjoint of a per-blade plan
// (one knot per blade); the volume gradient G_b flows back through the factors to the
// grids in gather form (no atomics), deterministic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vp {

constexpr int kKpMaxScales = 2;
enum { KP_XY = 0, KP_XS = 1, KP_YS = 2, KP_XT = 3, KP_YT = 4, KP_ST = 5, KP_PLANES = 6 };

struct KPDesc {
    int n, S, B, F, Rt, ns;                 // B: number of times (blades in a fit)
    int R[kKpMaxScales];
    long long off[kKpMaxScales][KP_PLANES];  // offsets of the grids in the flat vector
    long long a_off, n_params;
    // spatial interpolation, per scale: lower node and weight of each of the n samples,
    // and the transpose (per node: samples and weights, samples ascending)
    const int* nd0;      // [ns][n]
    const float* ndw;    // [ns][n]
    const int* tr_ptr;   // [ns][n + 1] (node j of scale c at c * (n + 1) + j)
    const int* tr_smp;   // samples
    const float* tr_w;   // weights
    // time interpolation per time b and its transpose (per node: times and weights)
    const int* tk;       // [B]
    const float* ta;     // [B]
    const int* tt_ptr;   // [R_t + 1]
    const int* tt_b;
    const float* tt_w;
    // parameters and their gradient
    const float2* params;
    float2* grad;
    // factors and their gradients
    float2 *Xs, *Ys;     // [ns][S][n][F]
    float2 *qx, *qy;     // [ns][B][n][F]
    float2* qs;          // [ns][B][S][F]
    float2* Z;           // [ns][n][n][F]
    float2 *XA, *Yf;     // [ns][B][S][n][F]
    float2 *gZ, *gY;
    float2* gXA;         // [2][ns][B][S][n][F]: row-range partial sums, summed into part 0
    float2* zpart;       // [zchunks][ns][n][n][F] partial sums of gZ over (b, s) chunks
    int zchunks;
    float2 *gXs, *gYs, *gqx, *gqy, *gqs, *h;  // h: [ns][B][S][F]
    float2* ga;          // [F]
    // dense per-blade volumes and their gradient [B][S][n][n]
    float2* vol;
    const float2* G;
    // optimiser
    float2 *m, *v;       // Adam moments of Re and Im per parameter
    int* step;           // device step counter (nullptr: step 0)
    int optimizer;
    float lr, beta1, beta2, c1, c2, aeps, ln_beta1, ln_beta2;
    // regularisers
    float tv_w, smooth_w, sparse_w, eps2;     // eps2 = max(eps^2, FLT_MIN)
    double* rpart;       // regulariser value partials, one per block of k_kp_reg_value
};

// Stages of one fit step (and of the gradient operator), in order.
hipError_t kp_launch_factors(const KPDesc& d, hipStream_t s);   // Xs, Ys, qx, qy, qs, Z, XA, Yf
hipError_t kp_launch_decode(const KPDesc& d, hipStream_t s);    // vol
hipError_t kp_launch_back(const KPDesc& d, hipStream_t s);      // gZ, gXA, gY from G
hipError_t kp_launch_back_z(const KPDesc& d, hipStream_t s);    // gZ
hipError_t kp_launch_back_x(const KPDesc& d, hipStream_t s);    // gXA
hipError_t kp_launch_back_y(const KPDesc& d, hipStream_t s);    // gY
hipError_t kp_launch_chain(const KPDesc& d, hipStream_t s);     // grid gradients + regulariser -> grad
hipError_t kp_launch_update(const KPDesc& d, hipStream_t s);    // Adam / GD on params (in place)
// Regulariser value: per-block FP64 partials into d.rpart; returns the block count.
int kp_reg_blocks(const KPDesc& d);
hipError_t kp_launch_reg_value(const KPDesc& d, hipStream_t s);
// proj / water / fat [B][n][n] from vol [B][S][n][n] (outputs may be null).
hipError_t kp_launch_render(const KPDesc& d, int split, float2* proj, float2* water, float2* fat, hipStream_t s);
bool kp_features_ok(int f);

}  // namespace vp
