// Blade-aligned sampling by gridding: kernel arguments and launchers (k_nu.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "vp_internal.h"

namespace vp {

struct NuArgs {
    int n, M, B, lmax, nparts;
    float kmax;             // bound on |kNuSigma k| over every sample (grid units)
    const int* lines;       // [B]
    const double2* cs;      // [B] (cos, sin) of the blade angle, FP64
    const float* dea;       // [n] 1 / (kernel transform) at the centred index x - n/2
    const float* kb;        // [kNuTable + 1] kernel on [0, W/2]
    const float2* ph;       // [B][lmax][n] exp(-i pi (kx + ky) 2 floor(n/2) / n) / n
    const BladeDev* blade;  // knot blend of dynamic blades (forward row pass)
    const float2* work;     // projection parts [B][nparts][n][n] (forward row pass)
    float2* img_out;        // adjoint images, part 0 of [B][nparts][n][n] (inverse row pass)
    float2* grid;           // oversampled grids [B][M][M]
    const float2* y;        // measured samples [B][lmax][n] (interp; may be null)
    float2* out;            // samples [B][lmax][n] (interp)
    const float2* s_in;     // samples [B][lmax][n] (prep)
    float2* pre;            // [B][lmax][n] dw conj(phase) times the samples the spread takes:
                            // written by interp (of its residual, when not null) or prep
    float dw;               // data-term weight of a fit; 1 for the operator
    float* loss;            // per-block sums of |out|^2 (interp with loss), or null
    // one-blade schedules of a fit: interp and spread skip the blades that are not active
    // at the device step counter (all blades when stepp is null or sched is all-blades)
    int sched;
    unsigned sseed;
    const int* stepp;
};

hipError_t nu_launch_interp(const NuArgs& d, hipStream_t s);
// Blocks of the interpolation launch (the length of d.loss).
int nu_interp_blocks(const NuArgs& d);
// pre = dw conj(phase) s_in (the adjoint operator's input to the spread)
hipError_t nu_launch_prep(const NuArgs& d, hipStream_t s);
hipError_t nu_launch_spread(const NuArgs& d, hipStream_t s);

}  // namespace vp
