// Blade-aligned (non-Cartesian) k-space sampling by gridding: blade b's samples lie on its
// rotated lattice k = r u_b + q n_b (readout r = j - n/2, line q = l - L_b/2). Forward:
// the projected image, centred and divided by the Kaiser-Bessel kernel's transform, is
// zero-padded onto a grid oversampled by kNuSigma and DFT'd (the row and column passes
// of an oversampled plan; its forward row pass builds the padded rows from the blade
// image), and every sample interpolated from the W x W grid points around it. Adjoint:
// the same weights gathered back onto every grid point (the lattice makes the samples
// near a grid point enumerable, so no atomics), inverse DFT, crop and divide (the
// inverse row pass writes the divided centre back) (Beatty, Nishimura and Pauly 2005,
// for the kernel and its transform).

#include "kcommon.h"
#include "nu.h"

namespace vp {

namespace {

__device__ __forceinline__ long long gtid() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * blockDim.x; }

// Kernel value at offset u (grid units) from the table over [0, W/2]; 0 beyond W/2 (and
// for NaN). Branch-free, so the loads of several lookups and of the data they weigh
// can be in flight together.
__device__ __forceinline__ float kb(const float* tab, float u) {
    const float a = fabsf(u) * ((float)kNuTable / (0.5f * kNuWidth));
    const bool in = a <= (float)kNuTable;
    const float ac = in ? a : 0.f;
    const int i = min((int)ac, kNuTable - 1);
    const float v = __builtin_fmaf(ac - (float)i, tab[i + 1] - tab[i], tab[i]);
    return in ? v : 0.f;
}

__device__ __forceinline__ int wrap(int m, int M) { return ((m % M) + M) % M; }

// Sample (j, l) of blade b in grid units: kNuSigma (r u_b + q n_b), r = j - n/2,
// q = l - L_b/2, in FP64 (exact to far below FP32's rounding of an offset). The
// interpolation and the spread evaluate this same expression, so a (sample, grid point)
// pair gets the same offsets, the same inclusion test and the same weights in both.
__device__ __forceinline__ double2 sample_pos(double2 cs, int j, int l, int n, int L) {
    const double r = (double)j - 0.5 * (double)n, q = (double)l - 0.5 * (double)L;
    return make_double2((double)kNuSigma * (r * cs.x - q * cs.y), (double)kNuSigma * (r * cs.y + q * cs.x));
}

// Grid points m0..m1 along one axis with |g - m| <= h as evaluated in FP64 (the test the
// spread applies): ceil/floor of g -+ h, moved by one where rounding puts them off.
__device__ __forceinline__ void axis_window(double g, double h, int& m0, int& m1) {
    m0 = (int)ceil(g - h);
    m1 = (int)floor(g + h);
    if (fabs(g - (double)(m0 - 1)) <= h) --m0;
    else if (fabs(g - (double)m0) > h) ++m0;
    if (fabs(g - (double)(m1 + 1)) <= h) ++m1;
    else if (fabs(g - (double)m1) > h) --m1;
}

// Lanes per sample in k_nu_interp: one per grid row of the window (at most 7 rows).
constexpr int kRowLanes = 8;
constexpr int kSamplesPerBlock = kThreads / kRowLanes;

// out[b][l][j] = (sum over the grid points within W/2 of 2k of C C grid) * phase / n - y.
// Each sample has kRowLanes lanes; lane r sums the window's r-th grid row (and r + 8, ...)
// times its row weight, and the sample's first lane adds the lanes' partials in lane
// order. With d.loss, each block also writes the sum of |out|^2 over its samples (fixed
// order).
__global__ __launch_bounds__(kThreads) void k_nu_interp(const NuArgs d) {
    __shared__ float2 part[kThreads];
    __shared__ float red[kThreads];
    float lsum = 0.f;
    const int n = d.n, M = d.M;
    const long long per = (long long)d.lmax * n;
    const long long total = (long long)d.B * per;
    const double h = 0.5 * (double)kNuWidth;
    const int sub = threadIdx.x % kRowLanes, slot = threadIdx.x / kRowLanes;
    const int st = read_step(d.stepp);
    // block-uniform loop: every lane reaches every barrier
    for (long long base = (long long)blockIdx.x * kSamplesPerBlock; base < total;
         base += (long long)gridDim.x * kSamplesPerBlock) {
        const long long e = base + slot;
        int L = 0, b = 0, l = 0, j = 0;
        if (e < total) {
            b = (int)(e / per);
            l = (int)((e % per) / n);
            j = (int)(e % n);
            L = d.lines[b];
        }
        float2 acc = make_float2(0.f, 0.f);
        const bool act = e < total && active_blade(d.sched, d.sseed, d.stepp, st, d.B, b);
        if (act && l < L) {
            const double2 g = sample_pos(d.cs[b], j, l, n, L);
            int x0, x1, y0, y1;
            axis_window(g.x, h, x0, x1);
            axis_window(g.y, h, y0, y1);
            const float2* grid = d.grid + (long long)b * M * M;
            for (int my = y0 + sub; my <= y1; my += kRowLanes) {
                const float cy = kb(d.kb, (float)(g.y - (double)my));
                const float2* row = grid + (long long)wrap(my, M) * M;
                float2 r = make_float2(0.f, 0.f);
                for (int mx = x0; mx <= x1; ++mx) r = cfma(kb(d.kb, (float)(g.x - (double)mx)), row[wrap(mx, M)], r);
                acc = cfma(cy, r, acc);
            }
        }
        part[threadIdx.x] = acc;
        __syncthreads();
        if (sub == 0 && e < total) {
            float2 v = make_float2(0.f, 0.f), w = v;
            if (act && l < L) {
#pragma unroll
                for (int r = 0; r < kRowLanes; ++r) v = cadd(v, part[threadIdx.x + r]);
                const float2 p = d.ph[e];
                v = cmul(v, p);
                if (d.y) v = csub(v, d.y[e]);
                w = cscale(cmul(v, make_float2(p.x, -p.y)), d.dw);
            }
            d.out[e] = v;
            if (d.pre) d.pre[e] = w;
            lsum = __builtin_fmaf(v.x, v.x, __builtin_fmaf(v.y, v.y, lsum));
        }
        __syncthreads();
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

// Readout range [lo, hi] of line q whose samples can lie within H (lattice units) of
// (X, Y) along one grid axis: |r a + q b - Z| <= H with (a, b) = (c, -s) for x and
// (s, c) for y (ia = 1/a). Returns false when no r can.
__device__ __forceinline__ bool axis_range(double a, double ia, double bq, double Z, double H, double& lo,
                                           double& hi) {
    if (fabs(a) < 1e-12) return fabs(bq - Z) <= H + 1e-9;
    const double u = (Z - bq - H) * ia, w = (Z - bq + H) * ia;
    lo = fmax(lo, fmin(u, w));
    hi = fmin(hi, fmax(u, w));
    return true;
}

// grid[b][gy][gx] = sum over the samples within W/2 (in both axes) of 2k - (gx, gy), at
// every wrap of the grid point, of C C s conj(phase): the transpose of k_nu_interp. The
// samples near a point are found from the lattice: the lines within reach, and on each
// the readout interval that meets both axis windows.
__global__ __launch_bounds__(kThreads) void k_nu_spread(const NuArgs d) {
    const int n = d.n, M = d.M;
    const long long MM = (long long)M * M;
    const long long total = (long long)d.B * MM;
    const double h = 0.5 * (double)kNuWidth;
    const double H = h / (double)kNuSigma;  // the window's half-width in lattice units
    const int st = read_step(d.stepp);
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / MM);
        // an inactive blade's grid is never read (its inverse passes and gather skip it)
        if (!active_blade(d.sched, d.sseed, d.stepp, st, d.B, b)) continue;
        const int py = (int)((e % MM) / M), px = (int)(e % M);
        const double2 cs = d.cs[b];
        const double c = cs.x, s = cs.y;
        const double ic = fabs(c) < 1e-12 ? 0.0 : 1.0 / c, is = fabs(s) < 1e-12 ? 0.0 : 1.0 / s;
        const int L = d.lines[b];
        const double qh = H * (fabs(c) + fabs(s)) + 1e-9;
        const float2* sv = d.pre + (long long)b * d.lmax * n;
        float2 acc = make_float2(0.f, 0.f);
        for (int ty = -1; ty <= 1; ++ty) {
            const int Py = py + ty * M;
            if ((float)abs(Py) > d.kmax + (float)h) continue;
            for (int tx = -1; tx <= 1; ++tx) {
                const int Px = px + tx * M;
                if ((float)abs(Px) > d.kmax + (float)h) continue;
                const double X = (double)Px / (double)kNuSigma, Y = (double)Py / (double)kNuSigma;
                const double q0 = -X * s + Y * c + 0.5 * (double)L;  // line index of the point
                const int l0 = max(0, (int)ceil(q0 - qh)), l1 = min(L - 1, (int)floor(q0 + qh));
                for (int l = l0; l <= l1; ++l) {
                    const double q = (double)l - 0.5 * (double)L;
                    double lo = -1e30, hi = 1e30;
                    if (!axis_range(c, ic, -q * s, X, H, lo, hi) || !axis_range(s, is, q * c, Y, H, lo, hi)) continue;
                    const int j0 = max(0, (int)ceil(lo + 0.5 * (double)n - 1e-9));
                    const int j1 = min(n - 1, (int)floor(hi + 0.5 * (double)n + 1e-9));
                    for (int j = j0; j <= j1; ++j) {
                        const double2 g = sample_pos(cs, j, l, n, L);
                        const double dx = g.x - (double)Px, dy = g.y - (double)Py;
                        if (fabs(dx) <= h && fabs(dy) <= h) {
                            acc = cfma(kb(d.kb, (float)dy) * kb(d.kb, (float)dx), sv[l * n + j], acc);
                        }
                    }
                }
            }
        }
        d.grid[e] = acc;
    }
}

// pre[b][l][j] = dw conj(phase) s_in (0 on lines l >= L_b)
__global__ __launch_bounds__(kThreads) void k_nu_prep(const NuArgs d) {
    const long long per = (long long)d.lmax * d.n;
    const long long total = (long long)d.B * per;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int b = (int)(e / per), l = (int)((e % per) / d.n);
        float2 w = make_float2(0.f, 0.f);
        if (l < d.lines[b]) {
            const float2 p = d.ph[e];
            w = cscale(cmul(d.s_in[e], make_float2(p.x, -p.y)), d.dw);
        }
        d.pre[e] = w;
    }
}

inline unsigned grid_of(long long total) {
    const long long g = (total + kThreads - 1) / kThreads;
    return (unsigned)(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

}  // namespace

int nu_interp_blocks(const NuArgs& d) { return (int)grid_of((long long)d.B * d.lmax * d.n * kRowLanes); }
hipError_t nu_launch_interp(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_interp, dim3(nu_interp_blocks(d)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t nu_launch_prep(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_prep, dim3(grid_of((long long)d.B * d.lmax * d.n)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t nu_launch_spread(const NuArgs& d, hipStream_t s) {
    hipLaunchKernelGGL(k_nu_spread, dim3(grid_of((long long)d.B * d.M * d.M)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}

}  // namespace vp
