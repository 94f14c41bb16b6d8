// Blade-aligned (non-Cartesian) k-space sampling by gridding: blade b's samples lie on its
// rotated lattice k = r u_b + q n_b (readout r = j - n/2, line q = l - L_b/2). Forward:
// the projected image, centred and divided by the Kaiser-Bessel kernel's transform, is
// zero-padded onto a grid oversampled by kNuSigma, DFT'd (the plan's row and column
// passes on the oversampled grid), and every sample interpolated from the W x W grid
// points around it. Adjoint: the same weights gathered back onto every grid point (the
// lattice makes the samples near a grid point enumerable, so no atomics), inverse DFT,
// crop and divide (Beatty, Nishimura and Pauly 2005, for the kernel and its transform).

#include "kcommon.h"
#include "nu.h"

namespace vp {

namespace {

__device__ __forceinline__ long long gtid() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * blockDim.x; }

// Kernel value at offset u (grid units) from the table over [0, W/2]; 0 beyond W/2.
__device__ __forceinline__ float kb(const float* tab, float u) {
    const float a = fabsf(u) * ((float)kNuTable / (0.5f * kNuWidth));
    if (!(a <= (float)kNuTable)) return 0.f;
    const int i = min((int)a, kNuTable - 1);
    return __builtin_fmaf(a - (float)i, tab[i + 1] - tab[i], tab[i]);
}

__device__ __forceinline__ int wrap(int m, int M) { return ((m % M) + M) % M; }

// Image index of oversampled grid index g (centred image, wrapped), or -1.
__device__ __forceinline__ int img_index(int g, int n, int M) {
    const int h = n / 2;
    if (g < n - h) return g + h;
    if (g >= M - h) return g - M + h;
    return -1;
}

// pad[b][gy][gx] = P_b[y][x] / (c(x) c(y)) at the centred, wrapped position; P_b blends a
// dynamic blade's two knot projections.
__global__ __launch_bounds__(kThreads) void k_nu_pad(const NuArgs d) {
    const int n = d.n, M = d.M;
    const long long MM = (long long)M * M, nn = (long long)n * n;
    const long long total = (long long)d.B * MM;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / MM);
        const int gy = (int)((e % MM) / M), gx = (int)(e % M);
        const int x = img_index(gx, n, M), y = img_index(gy, n, M);
        float2 v = make_float2(0.f, 0.f);
        if (x >= 0 && y >= 0) {
            const float2* p = d.work + (long long)b * d.nparts * nn + (long long)y * n + x;
            if (d.nparts == 2) {
                const BladeDev bd = d.blade[b];
                if (bd.has0) v = cscale(p[0], bd.w0);
                if (bd.has1) v = cfma(bd.w1, p[nn], v);
            } else {
                v = p[0];
            }
            v = cscale(v, d.dea[x] * d.dea[y]);
        }
        d.grid[e] = v;
    }
}

// out[b][l][j] = (sum over the grid points within W/2 of 2k of C C grid) * phase / n - y;
// with d.loss, each block also writes the sum of |out|^2 over its samples (fixed order)
__global__ __launch_bounds__(kThreads) void k_nu_interp(const NuArgs d) {
    __shared__ float red[kThreads];
    float lsum = 0.f;
    const int n = d.n, M = d.M;
    const long long per = (long long)d.lmax * n;
    const long long total = (long long)d.B * per;
    const float h = 0.5f * kNuWidth;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / per);
        const int l = (int)((e % per) / n);
        float2 v = make_float2(0.f, 0.f);
        if (l < d.lines[b]) {
            // offsets to grid point m: (kg - m) + kf, exact integer plus fraction
            const int2 kg = d.kg[e];
            const float2 kf = d.kf[e];
            const int x0 = kg.x + (int)ceilf(kf.x - h), x1 = kg.x + (int)floorf(kf.x + h);
            const int y0 = kg.y + (int)ceilf(kf.y - h), y1 = kg.y + (int)floorf(kf.y + h);
            const float2* g = d.grid + (long long)b * M * M;
            for (int my = y0; my <= y1; ++my) {
                const float cy = kb(d.kb, (float)(kg.y - my) + kf.y);
                const float2* row = g + (long long)wrap(my, M) * M;
                float2 r = make_float2(0.f, 0.f);
                for (int mx = x0; mx <= x1; ++mx) r = cfma(kb(d.kb, (float)(kg.x - mx) + kf.x), row[wrap(mx, M)], r);
                v = cfma(cy, r, v);
            }
            v = cmul(v, d.ph[e]);
            if (d.y) v = csub(v, d.y[e]);
        }
        d.out[e] = v;
        lsum = __builtin_fmaf(v.x, v.x, __builtin_fmaf(v.y, v.y, lsum));
    }
    if (d.loss) {
        red[threadIdx.x] = lsum;
        __syncthreads();
        for (int hh = kThreads / 2; hh > 0; hh >>= 1) {
            if ((int)threadIdx.x < hh) red[threadIdx.x] += red[threadIdx.x + hh];
            __syncthreads();
        }
        if (threadIdx.x == 0) d.loss[blockIdx.x] = red[0];
    }
}

// grid[b][gy][gx] = sum over the samples within W/2 (in both axes) of 2k - (gx, gy), at
// every wrap of the grid point, of C C s conj(phase): the transpose of k_nu_interp.
__global__ __launch_bounds__(kThreads) void k_nu_spread(const NuArgs d) {
    const int n = d.n, M = d.M;
    const long long MM = (long long)M * M;
    const long long total = (long long)d.B * MM;
    const float h = 0.5f * kNuWidth;
    // lattice half-window: the W x W box around a grid point, in lattice units
    const float hw = h / (float)kNuSigma * 1.41421356f + 1e-3f;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / MM);
        const int py = (int)((e % MM) / M), px = (int)(e % M);
        const float c = d.cs[b].x, s = d.cs[b].y;
        const int L = d.lines[b];
        const int2* kg = d.kg + (long long)b * d.lmax * n;
        const float2* kf = d.kf + (long long)b * d.lmax * n;
        const float2* sv = d.s_in + (long long)b * d.lmax * n;
        const float2* ph = d.ph + (long long)b * d.lmax * n;
        float2 acc = make_float2(0.f, 0.f);
        for (int ty = -1; ty <= 1; ++ty) {
            const int Py = py + ty * M;
            if ((float)abs(Py) > d.kmax + h) continue;
            for (int tx = -1; tx <= 1; ++tx) {
                const int Px = px + tx * M;
                if ((float)abs(Px) > d.kmax + h) continue;
                const float kx = (float)Px / (float)kNuSigma, ky = (float)Py / (float)kNuSigma;
                const float r0 = kx * c + ky * s + 0.5f * (float)n;   // readout index of the point
                const float q0 = -kx * s + ky * c + 0.5f * (float)L;  // line index of the point
                const int j0 = max(0, (int)ceilf(r0 - hw)), j1 = min(n - 1, (int)floorf(r0 + hw));
                const int l0 = max(0, (int)ceilf(q0 - hw)), l1 = min(L - 1, (int)floorf(q0 + hw));
                for (int l = l0; l <= l1; ++l) {
                    for (int j = j0; j <= j1; ++j) {
                        const long long i = (long long)l * n + j;
                        // the offsets k_nu_interp weighs this pair with, bit for bit
                        const int2 g = kg[i];
                        const float2 f = kf[i];
                        const float dx = (float)(g.x - Px) + f.x;
                        const float dy = (float)(g.y - Py) + f.y;
                        if (fabsf(dx) <= h && fabsf(dy) <= h) {
                            const float2 p = ph[i];
                            const float2 v = cscale(cmul(sv[i], make_float2(p.x, -p.y)), d.dw);
                            acc = cfma(kb(d.kb, dy) * kb(d.kb, dx), v, acc);
                        }
                    }
                }
            }
        }
        d.grid[e] = acc;
    }
}

// img[b][y][x] (work part 0) = grid at the wrapped centred position / (c(x) c(y))
__global__ __launch_bounds__(kThreads) void k_nu_crop(const NuArgs d) {
    const int n = d.n, M = d.M, hh = n / 2;
    const long long nn = (long long)n * n;
    const long long total = (long long)d.B * nn;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / nn);
        const int y = (int)((e % nn) / n), x = (int)(e % n);
        const int gx = wrap(x - hh, M), gy = wrap(y - hh, M);
        const float2 v = d.grid[((long long)b * M + gy) * M + gx];
        d.img_out[(long long)b * d.nparts * nn + (long long)y * n + x] = cscale(v, d.dea[x] * d.dea[y]);
    }
}

inline unsigned grid_of(long long total) {
    const long long g = (total + kThreads - 1) / kThreads;
    return (unsigned)(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

}  // namespace

hipError_t nu_launch_pad(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_pad, dim3(grid_of((long long)d.B * d.M * d.M)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
int nu_interp_blocks(const NuArgs& d) { return (int)grid_of((long long)d.B * d.lmax * d.n); }
hipError_t nu_launch_interp(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_interp, dim3(nu_interp_blocks(d)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t nu_launch_spread(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_spread, dim3(grid_of((long long)d.B * d.M * d.M)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t nu_launch_crop(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_crop, dim3(grid_of((long long)d.B * d.n * d.n)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}

}  // namespace vp
