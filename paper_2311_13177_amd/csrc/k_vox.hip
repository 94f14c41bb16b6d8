// Voxel-wise kernels: operator TV/L1 gradient, objective regulariser terms and the
// renders (Section 4.3, Section 6 fat/water split).

#include "kcommon.h"

namespace vp {

// tv_w * grad TV + l1_w * grad L1 at voxel (t, s, y, x) of a [T][S][n][n] volume.
__device__ __forceinline__ float2 reg_grad(const float2* __restrict__ V, size_t idx, int t, int s, int y, int x,
                                           int n, int S, int T, float tv_w, float l1_w, float eps) {
    const float eps2 = charb_eps2(eps);
    const float2 v0 = V[idx];
    float2 g = make_float2(0.f, 0.f);
    if (tv_w != 0.f) {
        const size_t nn = (size_t)n * n;
        if (t > 0) g = cadd(g, charb_w(csub(v0, V[idx - (size_t)S * nn]), eps2));
        if (t + 1 < T) g = csub(g, charb_w(csub(V[idx + (size_t)S * nn], v0), eps2));
        if (s > 0) g = cadd(g, charb_w(csub(v0, V[idx - nn]), eps2));
        if (s + 1 < S) g = csub(g, charb_w(csub(V[idx + nn], v0), eps2));
        if (y > 0) g = cadd(g, charb_w(csub(v0, V[idx - n]), eps2));
        if (y + 1 < n) g = csub(g, charb_w(csub(V[idx + n], v0), eps2));
        if (x > 0) g = cadd(g, charb_w(csub(v0, V[idx - 1]), eps2));
        if (x + 1 < n) g = csub(g, charb_w(csub(V[idx + 1], v0), eps2));
        g = cscale(g, tv_w);
    }
    if (l1_w != 0.f) g = cfma(l1_w, charb_w(v0, eps2), g);
    return g;
}

// ------------------------------------------------------------------ voxel-wise kernels

// Operator TV/L1 gradient: grad (+)= tv_w grad TV + l1_w grad L1 (weights from the descriptor).
__global__ __launch_bounds__(kThreads) void k_tv_grad(const KArgs a) {
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        const int n = DF(n), S = DF(S), T = DF(T);
        const float tv_w = DF(tv_w), l1_w = DF(l1_w), teps = DF(tv_eps);
        const float2* V = DF(vol[0]);
        float2* grad = DF(grad);
        const size_t nvox = (size_t)T * S * n * n;
        const size_t i0 = (size_t)tk->a * kVoxItem;
        for (size_t i = i0 + threadIdx.x; i < min(nvox, i0 + kVoxItem); i += blockDim.x) {
            const int x = (int)(i % n), y = (int)((i / n) % n), s = (int)((i / ((size_t)n * n)) % S);
            const int t = (int)(i / ((size_t)S * n * n));
            float2 g = reg_grad(V, i, t, s, y, x, n, S, T, tv_w, l1_w, teps);
            if (a.accumulate) g = cadd(grad[i], g);
            grad[i] = g;
        }
    }
}

// Objective regulariser terms: per work item, sums of the TV terms (forward differences
// where the neighbour exists) and the L1 terms, each written as |z|^2 / (sqrt(|z|^2 + e^2) + e),
// the cancellation-free form of sqrt(|z|^2 + e^2) - e. Output a.dpart[2 * item + {0, 1}].
__global__ __launch_bounds__(kThreads) void k_reg_value(const KArgs a) {
    __shared__ double red[2][kThreads];
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        const int n = DF(n), S = DF(S), T = DF(T);
        const size_t nn = (size_t)n * n, nvox = (size_t)T * S * nn;
        const size_t i0 = (size_t)tk->a * kVoxItem;
        const float2* V = stepp ? DF(vol[st & 1]) : DF(vol[0]);
        const float e = DF(tv_eps), e2 = e * e;
        double tv = 0.0, l1 = 0.0;
        for (size_t i = i0 + threadIdx.x; i < min(nvox, i0 + kVoxItem); i += blockDim.x) {
            const int x = (int)(i % n), y = (int)((i / n) % n), s = (int)((i / nn) % S);
            const int t = (int)(i / ((size_t)S * nn));
            const float2 v0 = V[i];
            float part = 0.f;
            auto term = [&](float2 z) {
                const float q = __builtin_fmaf(z.x, z.x, z.y * z.y);
                return q / (sqrtf(q + e2) + e);
            };
            if (x + 1 < n) part += term(csub(V[i + 1], v0));
            if (y + 1 < n) part += term(csub(V[i + n], v0));
            if (s + 1 < S) part += term(csub(V[i + nn], v0));
            if (t + 1 < T) part += term(csub(V[i + (size_t)S * nn], v0));
            tv += part;
            l1 += term(v0);
        }
        red[0][threadIdx.x] = tv;
        red[1][threadIdx.x] = l1;
        __syncthreads();
        for (int w = kThreads / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) {
                red[0][threadIdx.x] += red[0][threadIdx.x + w];
                red[1][threadIdx.x] += red[1][threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            a.dpart[2 * ti] = red[0][0];
            a.dpart[2 * ti + 1] = red[1][0];
        }
        __syncthreads();
    }
}

// Render at phi = 0 and the fat/water split: water = bins [0, split), fat = [split, S),
// proj = water + fat. One work item per (knot, block of kVoxItem pixels).
__global__ __launch_bounds__(kThreads) void k_render(const KArgs a) {
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        const int n = DF(n), S = DF(S);
        const size_t nn = (size_t)n * n;
        const int split = a.split_bin < 0 ? S / 2 : min(a.split_bin, S);
        const float2* V = (stepp ? DF(vol[st & 1]) : DF(vol[0])) + (size_t)tk->a * S * nn;
        const size_t p0 = (size_t)tk->b * kVoxItem;
        for (size_t p = p0 + threadIdx.x; p < min(nn, p0 + kVoxItem); p += blockDim.x) {
            float2 w = make_float2(0.f, 0.f), f = make_float2(0.f, 0.f);
            for (int s = 0; s < split; ++s) w = cadd(w, V[(size_t)s * nn + p]);
            for (int s = split; s < S; ++s) f = cadd(f, V[(size_t)s * nn + p]);
            const size_t o = (size_t)tk->a * nn + p;
            if (a.out0) a.out0[o] = cadd(w, f);
            if (a.out1) a.out1[o] = w;
            if (a.out2) a.out2[o] = f;
        }
    }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int ntasks) { return ntasks < 1 ? 1 : (ntasks > (1 << 20) ? (1 << 20) : ntasks); }

hipError_t launch_tv_grad(const KArgs& a, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tv_grad, dim3(grid_for(a.ntasks)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_reg_value(const KArgs& a, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reg_value, dim3(grid_for(a.ntasks)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_render(const KArgs& a, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_render, dim3(grid_for(a.ntasks)), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace vp
