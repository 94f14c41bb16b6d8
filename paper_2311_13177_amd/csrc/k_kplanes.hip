// Kernels of the complex K-Planes dynamic model (Section 4.1): the separable factors,
// the dense per-blade decode, the gradient back through the factors (gather form, fixed
// summation orders), the grid regularisers of Section 4.3 and the optimiser update.

#include "kcommon.h"
#include "kplanes.h"

namespace vp {

namespace {

// a * b + c and conj(a) * b + c with explicit fused multiply-adds
__device__ __forceinline__ float2 cmad(float2 a, float2 b, float2 c) {
    return make_float2(__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, c.x)),
                       __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 cjmad(float2 a, float2 b, float2 c) {
    return make_float2(__builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, c.x)),
                       __builtin_fmaf(a.x, b.y, __builtin_fmaf(-a.y, b.x, c.y)));
}
// (1 - w) a + w b
__device__ __forceinline__ float2 clerp(float2 a, float2 b, float w) { return cfma(w, b, cscale(a, 1.0f - w)); }

__device__ __forceinline__ long long gtid() { return (long long)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ long long gstride() { return (long long)gridDim.x * blockDim.x; }

// Grid value of scale c along one spatial axis at sample i: p[stride * node] rows.
__device__ __forceinline__ float2 read_x(const float2* p, long long stride, const KPDesc& d, int c, int i) {
    const int i0 = d.nd0[c * d.n + i];
    const int i1 = min(i0 + 1, d.R[c] - 1);
    return clerp(p[i0 * stride], p[i1 * stride], d.ndw[c * d.n + i]);
}

// ------------------------------------------------------------------ factors

// Xs, Ys [ns][S][n][F]
__global__ __launch_bounds__(kThreads) void k_kp_fac_s(const KPDesc d) {
    const long long total = (long long)d.ns * d.S * d.n * d.F;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int f = (int)(e % d.F);
        const int i = (int)((e / d.F) % d.n);
        const int s = (int)((e / ((long long)d.F * d.n)) % d.S);
        const int c = (int)(e / ((long long)d.F * d.n * d.S));
        const int R = d.R[c];
        const float2* xs = d.params + d.off[c][KP_XS] + (long long)s * R * d.F + f;
        const float2* ys = d.params + d.off[c][KP_YS] + (long long)s * R * d.F + f;
        d.Xs[e] = read_x(xs, d.F, d, c, i);
        d.Ys[e] = read_x(ys, d.F, d, c, i);
    }
}

// qx, qy [ns][B][n][F] and qs [ns][B][S][F]: time grids at each time
__global__ __launch_bounds__(kThreads) void k_kp_fac_t(const KPDesc d) {
    const long long nq = (long long)d.ns * d.B * d.n * d.F;
    const long long total = nq + (long long)d.ns * d.B * d.S * d.F;
    for (long long e = gtid(); e < total; e += gstride()) {
        if (e < nq) {
            const int f = (int)(e % d.F);
            const int i = (int)((e / d.F) % d.n);
            const int b = (int)((e / ((long long)d.F * d.n)) % d.B);
            const int c = (int)(e / ((long long)d.F * d.n * d.B));
            const int R = d.R[c];
            const int k0 = d.tk[b], k1 = min(k0 + 1, d.Rt - 1);
            const float a = d.ta[b];
            const float2* xt = d.params + d.off[c][KP_XT] + f;
            const float2* yt = d.params + d.off[c][KP_YT] + f;
            const long long row = (long long)R * d.F;
            d.qx[e] = clerp(read_x(xt + k0 * row, d.F, d, c, i), read_x(xt + k1 * row, d.F, d, c, i), a);
            d.qy[e] = clerp(read_x(yt + k0 * row, d.F, d, c, i), read_x(yt + k1 * row, d.F, d, c, i), a);
        } else {
            const long long r = e - nq;
            const int f = (int)(r % d.F);
            const int s = (int)((r / d.F) % d.S);
            const int b = (int)((r / ((long long)d.F * d.S)) % d.B);
            const int c = (int)(r / ((long long)d.F * d.S * d.B));
            const int k0 = d.tk[b], k1 = min(k0 + 1, d.Rt - 1);
            const float2* st = d.params + d.off[c][KP_ST] + (long long)s * d.F + f;
            const long long row = (long long)d.S * d.F;
            d.qs[r] = clerp(st[k0 * row], st[k1 * row], d.ta[b]);
        }
    }
}

// Z [ns][n][n][F]: the xy grid at (y, x), along x first
__global__ __launch_bounds__(kThreads) void k_kp_fac_z(const KPDesc d) {
    const long long total = (long long)d.ns * d.n * d.n * d.F;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int f = (int)(e % d.F);
        const int x = (int)((e / d.F) % d.n);
        const int y = (int)((e / ((long long)d.F * d.n)) % d.n);
        const int c = (int)(e / ((long long)d.F * d.n * d.n));
        const int R = d.R[c];
        const float2* xy = d.params + d.off[c][KP_XY] + f;
        const int j0 = d.nd0[c * d.n + y], j1 = min(j0 + 1, R - 1);
        const float2 r0 = read_x(xy + (long long)j0 * R * d.F, d.F, d, c, x);
        const float2 r1 = read_x(xy + (long long)j1 * R * d.F, d.F, d, c, x);
        d.Z[e] = clerp(r0, r1, d.ndw[c * d.n + y]);
    }
}

// XA = a Xs qx qs and Yf = Ys qy, [ns][B][S][n][F]
__global__ __launch_bounds__(kThreads) void k_kp_prod(const KPDesc d) {
    const long long total = (long long)d.ns * d.B * d.S * d.n * d.F;
    for (long long e = gtid(); e < total; e += gstride()) {
        const int f = (int)(e % d.F);
        const int i = (int)((e / d.F) % d.n);
        const int s = (int)((e / ((long long)d.F * d.n)) % d.S);
        const int b = (int)((e / ((long long)d.F * d.n * d.S)) % d.B);
        const int c = (int)(e / ((long long)d.F * d.n * d.S * d.B));
        const long long xs = (((long long)c * d.S + s) * d.n + i) * d.F + f;
        const long long qi = (((long long)c * d.B + b) * d.n + i) * d.F + f;
        const long long qsi = (((long long)c * d.B + b) * d.S + s) * d.F + f;
        const float2 a = d.params[d.a_off + f];
        d.XA[e] = cmul(cmul(cmul(a, d.Xs[xs]), d.qx[qi]), d.qs[qsi]);
        d.Yf[e] = cmul(d.Ys[xs], d.qy[qi]);
    }
}

// ------------------------------------------------------------------ decode

// vol[b][s][y][x] = sum_c sum_f Z[c][y][x][f] XA[c][b][s][x][f] Yf[c][b][s][y][f]
constexpr int kDecBins = 4;

// Values that are the same for a whole wave are loaded spread over its lanes, one vector
// load for up to 64 of them, and read back with lane_f2.
constexpr int kDecRows = 4;

// A wave task is (blade, kDecBins bins, kDecRows rows, 64 columns): its XA values (per
// column) are loaded once for all kDecRows rows, its Yf values (per row, the same in
// every lane) once for the wave spread over the lanes, and Z (per pixel) once per row for
// all kDecBins bins. The sums run in the same order as a per-voxel loop (scales, then
// features), so every shape of this task gives the same bits.
template <int F>
__global__ __launch_bounds__(kThreads) void k_kp_decode(const KPDesc d) {
    constexpr int NY = kDecRows * kKpMaxScales * kDecBins * F;  // Yf entries of one wave task
    constexpr int NL = (NY + 63) / 64;
    const int n = d.n, S = d.S;
    const long long nn = (long long)n * n;
    const int sq = (S + kDecBins - 1) / kDecBins;
    const int nseg = (n + 63) / 64, nrg = (n + kDecRows - 1) / kDecRows;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long W = (long long)d.B * sq * nrg * nseg;
    for (long long w = (long long)blockIdx.x * (kThreads / 64) + wave; w < W; w += (long long)gridDim.x * (kThreads / 64)) {
        const int seg = (int)(w % nseg);
        const int rg = (int)((w / nseg) % nrg);
        const int q = (int)((w / ((long long)nseg * nrg)) % sq);
        const int b = (int)(w / ((long long)nseg * nrg * sq));
        const int s0 = q * kDecBins, ns = min(kDecBins, S - s0);
        const int y0 = rg * kDecRows;
        // Yf of the task, one entry per lane: ((r kKpMaxScales + c) kDecBins + k) F + f
        float2 yl[NL];
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int ei = t * 64 + lane;
            const int f = ei % F, k = (ei / F) % kDecBins, c = (ei / (F * kDecBins)) % kKpMaxScales;
            const int r = ei / (F * kDecBins * kKpMaxScales);
            yl[t] = make_float2(0.f, 0.f);
            if (ei < NY && c < d.ns && k < ns && y0 + r < n)
                yl[t] = d.Yf[((((long long)c * d.B + b) * S + s0 + k) * n + y0 + r) * F + f];
        }
        const int x = seg * 64 + lane;
        const bool live = x < n;
        const int xs = live ? x : 0;
        float2 v[kDecRows][kDecBins];
#pragma unroll
        for (int r = 0; r < kDecRows; ++r)
#pragma unroll
            for (int k = 0; k < kDecBins; ++k) v[r][k] = make_float2(0.f, 0.f);
#pragma unroll
        for (int c = 0; c < kKpMaxScales; ++c) {
            if (c < d.ns) {
                float2 xa[kDecBins][F];
#pragma unroll
                for (int k = 0; k < kDecBins; ++k) {
                    const long long cb = ((long long)c * d.B + b) * S + s0 + min(k, ns - 1);
                    const float2* xp = d.XA + (cb * n + xs) * F;
#pragma unroll
                    for (int f = 0; f < F; ++f) xa[k][f] = xp[f];
                }
#pragma unroll
                for (int r = 0; r < kDecRows; ++r) {
                    const int y = min(y0 + r, n - 1);
                    float2 z[F];
                    const float2* zp = d.Z + ((long long)c * nn + (long long)y * n + xs) * F;
#pragma unroll
                    for (int f = 0; f < F; ++f) z[f] = zp[f];
#pragma unroll
                    for (int k = 0; k < kDecBins; ++k) {
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            const int ei = ((r * kKpMaxScales + c) * kDecBins + k) * F + f;
                            v[r][k] = cmad(cmul(z[f], xa[k][f]), lane_f2(yl[ei / 64], ei % 64), v[r][k]);
                        }
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int r = 0; r < kDecRows; ++r)
#pragma unroll
                for (int k = 0; k < kDecBins; ++k)
                    if (k < ns && y0 + r < n) d.vol[((long long)b * S + s0 + k) * nn + (long long)(y0 + r) * n + x] = v[r][k];
        }
    }
}

// ------------------------------------------------------------------ gradient through the factors

// gZ[c][y][x][f] = sum_b sum_s conj(XA Yf) G[b][s][y][x], in two passes: partial sums over
// consecutive (b, s) chunks for every pixel and both scales (G read once), then the
// chunks summed in order. A wave task of the first pass is (chunk, kGzRows rows, 64
// columns): each XA value (per column) serves all kGzRows rows, and the Yf values (per
// row, the same in every lane) of 64 / (kGzRows kKpMaxScales F) consecutive (b, s) are
// loaded at once spread over the lanes. Each sum runs over (b, s) in order.
constexpr int kGzRows = 2;

template <int F>
__global__ __launch_bounds__(kThreads) void k_kp_grad_z(const KPDesc d) {
    constexpr int NYB = kGzRows * kKpMaxScales * F;  // Yf entries per (b, s)
    constexpr int BPL = NYB >= 64 ? 1 : 64 / NYB;     // (b, s) per lane-spread load
    const int n = d.n;
    const long long nn = (long long)n * n;
    const int nbs = d.B * d.S, cs = (nbs + d.zchunks - 1) / d.zchunks;
    const int nseg = (n + 63) / 64, nrg = (n + kGzRows - 1) / kGzRows;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long W = (long long)d.zchunks * nrg * nseg;
    for (long long w = (long long)blockIdx.x * (kThreads / 64) + wave; w < W; w += (long long)gridDim.x * (kThreads / 64)) {
        const int seg = (int)(w % nseg);
        const int y0 = (int)((w / nseg) % nrg) * kGzRows;
        const int ch = (int)(w / ((long long)nseg * nrg));
        const int x = seg * 64 + lane;
        const bool live = x < n;
        const int xs = live ? x : 0;
        float2 acc[kGzRows][kKpMaxScales][F];
#pragma unroll
        for (int r = 0; r < kGzRows; ++r)
#pragma unroll
            for (int c = 0; c < kKpMaxScales; ++c)
#pragma unroll
                for (int f = 0; f < F; ++f) acc[r][c][f] = make_float2(0.f, 0.f);
        const int bs1 = min(nbs, (ch + 1) * cs);
        for (int bs = ch * cs; bs < bs1; bs += BPL) {
            float2 yl;
            {
                const int bq = bs + lane / NYB, ei = lane % NYB;
                const int r = ei / (kKpMaxScales * F), c = (ei / F) % kKpMaxScales, f = ei % F;
                yl = make_float2(0.f, 0.f);
                if (lane < BPL * NYB && bq < bs1 && c < d.ns && y0 + r < n)
                    yl = d.Yf[(((long long)c * nbs + bq) * n + y0 + r) * F + f];
            }
#pragma unroll
            for (int u = 0; u < BPL; ++u) {
                const int bu = bs + u;
                if (bu < bs1) {
                    float2 xa[kKpMaxScales][F];
#pragma unroll
                    for (int c = 0; c < kKpMaxScales; ++c) {
                        const float2* xp = d.XA + (((long long)min(c, d.ns - 1) * nbs + bu) * n + xs) * F;
#pragma unroll
                        for (int f = 0; f < F; ++f) xa[c][f] = xp[f];
                    }
#pragma unroll
                    for (int r = 0; r < kGzRows; ++r) {
                        if (y0 + r < n) {
                            const float2 g = d.G[(long long)bu * nn + (long long)(y0 + r) * n + xs];
#pragma unroll
                            for (int c = 0; c < kKpMaxScales; ++c) {
                                if (c < d.ns) {
#pragma unroll
                                    for (int f = 0; f < F; ++f)
                                        acc[r][c][f] = cjmad(cmul(xa[c][f], lane_f2(yl, u * NYB + (r * kKpMaxScales + c) * F + f)),
                                                             g, acc[r][c][f]);
                                }
                            }
                        }
                    }
                }
            }
        }
        if (live) {
#pragma unroll
            for (int r = 0; r < kGzRows; ++r) {
#pragma unroll
                for (int c = 0; c < kKpMaxScales; ++c) {
                    if (c < d.ns && y0 + r < n) {
                        float2* out = d.zpart + (((long long)ch * d.ns + c) * nn + (long long)(y0 + r) * n + x) * F;
#pragma unroll
                        for (int f = 0; f < F; ++f) out[f] = acc[r][c][f];
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_kp_grad_z_sum(const KPDesc d) {
    const long long per = (long long)d.ns * d.n * d.n * d.F;
    for (long long e = gtid(); e < per; e += gstride()) {
        float2 acc = make_float2(0.f, 0.f);
        for (int ch = 0; ch < d.zchunks; ++ch) acc = cadd(acc, d.zpart[(long long)ch * per + e]);
        d.gZ[e] = acc;
    }
}

// gXA[c][b][s][x][f] = sum_y conj(Z Yf) G[b][s][y][x]. A wave task is (kGxBs consecutive
// (b, s), 64 columns, one of kGxYs row ranges): each Z value (per pixel) serves all kGxBs
// (b, s), and the Yf values (per row, the same in every lane) are loaded 64 / F rows at a
// time spread over the lanes. The row split keeps the waves of one (b, s) per task while
// Z is shared; each range's sum runs over y in order into its own part of gXA, and
// k_kp_gx_sum adds the parts in order.
constexpr int kGxBs = 2;
constexpr int kGxYs = 2;  // row ranges

template <int F>
__global__ __launch_bounds__(kThreads) void k_kp_grad_x(const KPDesc d) {
    constexpr int YB = 64 / F;  // rows per lane-spread Yf load
    const int n = d.n;
    const long long nn = (long long)n * n;
    const int nbs = d.B * d.S;
    const int nseg = (n + 63) / 64, ngr = (nbs + kGxBs - 1) / kGxBs;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const long long W = (long long)ngr * nseg * kGxYs;
    const int rq = (n + kGxYs - 1) / kGxYs;
    for (long long w = (long long)blockIdx.x * (kThreads / 64) + wave; w < W; w += (long long)gridDim.x * (kThreads / 64)) {
        const int seg = (int)(w % nseg);
        const int half = (int)((w / nseg) % kGxYs);
        const int bs0 = (int)(w / ((long long)nseg * kGxYs)) * kGxBs;
        const int ya = min(n, half * rq), yb = min(n, ya + rq);
        const int x = seg * 64 + lane;
        const bool live = x < n;
        const int xs = live ? x : 0;
        for (int c = 0; c < d.ns; ++c) {
            float2 acc[kGxBs][F];
#pragma unroll
            for (int j = 0; j < kGxBs; ++j)
#pragma unroll
                for (int f = 0; f < F; ++f) acc[j][f] = make_float2(0.f, 0.f);
            for (int y0 = ya; y0 < yb; y0 += YB) {
                float2 yl[kGxBs];
                const int yy = y0 + lane / F;
#pragma unroll
                for (int j = 0; j < kGxBs; ++j) {
                    const int bs = bs0 + j;
                    yl[j] = make_float2(0.f, 0.f);
                    if (bs < nbs && yy < yb) yl[j] = d.Yf[(((long long)c * nbs + bs) * n + yy) * F + lane % F];
                }
#pragma unroll
                for (int t = 0; t < YB; ++t) {
                    const int y = y0 + t;
                    if (y < yb) {
                        float2 z[F];
                        const float2* zp = d.Z + (((long long)c * n + y) * n + xs) * F;
#pragma unroll
                        for (int f = 0; f < F; ++f) z[f] = zp[f];
#pragma unroll
                        for (int j = 0; j < kGxBs; ++j) {
                            if (bs0 + j < nbs) {
                                const float2 g = d.G[(long long)(bs0 + j) * nn + (long long)y * n + xs];
#pragma unroll
                                for (int f = 0; f < F; ++f)
                                    acc[j][f] = cjmad(cmul(z[f], lane_f2(yl[j], t * F + f)), g, acc[j][f]);
                            }
                        }
                    }
                }
            }
            if (live) {
#pragma unroll
                for (int j = 0; j < kGxBs; ++j) {
                    if (bs0 + j < nbs) {
                        float2* out = d.gXA + (long long)half * d.ns * nbs * n * F + (((long long)c * nbs + bs0 + j) * n + x) * F;
#pragma unroll
                        for (int f = 0; f < F; ++f) out[f] = acc[j][f];
                    }
                }
            }
        }
    }
}

// gXA (part 0) = the sum of the kGxYs row-range parts, in order
__global__ __launch_bounds__(kThreads) void k_kp_gx_sum(const KPDesc d) {
    const long long per = (long long)d.ns * d.B * d.S * d.n * d.F;
    for (long long e = gtid(); e < per; e += gstride()) {
        float2 v = d.gXA[e];
        for (int h = 1; h < kGxYs; ++h) v = cadd(v, d.gXA[h * per + e]);
        d.gXA[e] = v;
    }
}

// gY[c][b][s][y][f] = sum_x conj(Z XA) G[b][s][y][x]: one wave per block of 32 / F rows,
// RB consecutive (b, s) by RY consecutive y (each Z value serves the RB (b, s), each XA
// value the RY rows), lanes over x; the wave's 64 partial sums per lane (rows x features x
// re/im) are reduced across lanes by recursive halving, each step sending the half a lane
// gives up to its partner, so that lane L ends with the total of value L (a fixed order).
template <int F>
__global__ __launch_bounds__(kThreads) void k_kp_grad_y(const KPDesc d) {
    constexpr int RW = 32 / F;  // rows per wave: 2 F RW = 64 values
    constexpr int RY = RW >= 16 ? 4 : (RW >= 4 ? 2 : 1);
    constexpr int RB = RW / RY;
    const int n = d.n;
    const int lane = threadIdx.x & 63;
    const int nbs = d.B * d.S;
    const long long nyb = (n + RY - 1) / RY, nbb = (nbs + RB - 1) / RB;
    const long long groups = nbb * nyb;
    for (long long gi = (long long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); gi < groups;
         gi += (long long)gridDim.x * (kThreads / 64)) {
        const int y0 = (int)(gi % nyb) * RY;
        const int bs0 = (int)(gi / nyb) * RB;
        for (int c = 0; c < d.ns; ++c) {
            float v[64];
#pragma unroll
            for (int i = 0; i < 64; ++i) v[i] = 0.f;
            for (int x = lane; x < n; x += 64) {
                float2 zr[RY][F], xr[RB][F];
#pragma unroll
                for (int q = 0; q < RY; ++q) {
                    const float2* z = d.Z + (((long long)c * n + min(y0 + q, n - 1)) * n + x) * F;
#pragma unroll
                    for (int f = 0; f < F; ++f) zr[q][f] = z[f];
                }
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    const float2* xa = d.XA + (((long long)c * nbs + min(bs0 + q, nbs - 1)) * n + x) * F;
#pragma unroll
                    for (int f = 0; f < F; ++f) xr[q][f] = xa[f];
                }
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    const int rb = r / RY, ry = r % RY;
                    if (bs0 + rb < nbs && y0 + ry < n) {
                        const float2 g = d.G[((long long)(bs0 + rb) * n + y0 + ry) * n + x];
#pragma unroll
                        for (int f = 0; f < F; ++f) {
                            const float2 t = cjmad(cmul(zr[ry][f], xr[rb][f]), g,
                                                   make_float2(v[(r * F + f) * 2], v[(r * F + f) * 2 + 1]));
                            v[(r * F + f) * 2] = t.x;
                            v[(r * F + f) * 2 + 1] = t.y;
                        }
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const bool up = (lane & o) != 0;
#pragma unroll
                for (int i = 0; i < o; ++i) {
                    const float send = up ? v[i] : v[i + o];
                    const float keep = up ? v[i + o] : v[i];
                    v[i] = keep + __shfl_xor(send, o);
                }
            }
            // lane L holds value L: row L / (2F), feature (L / 2) % F, component L % 2
            const int r = lane / (2 * F), rb = r / RY, ry = r % RY;
            if (bs0 + rb < nbs && y0 + ry < n) {
                const long long cb = (long long)c * nbs + bs0 + rb;
                float* out = reinterpret_cast<float*>(d.gY + (cb * n + y0 + ry) * F);
                out[lane % (2 * F)] = v[0];
            }
        }
    }
}

// ------------------------------------------------------------------ chain to the grids

// Independent sums over one index each, a thread per output:
//   gXs[c][s][x][f] = sum_b conj(a qx qs) gXA        gqx[c][b][x][f] = sum_s conj(a Xs qs) gXA
//   gYs[c][s][y][f] = sum_b conj(qy) gY              gqy[c][b][y][f] = sum_s conj(Ys) gY
// (h and gqs, with far fewer outputs and a longer sum, are k_kp_chain_h's)
__global__ __launch_bounds__(kThreads) void k_kp_chain1(const KPDesc d) {
    const int n = d.n, S = d.S, B = d.B, F = d.F;
    const long long n_sn = (long long)d.ns * S * n * F;   // gXs, gYs
    const long long n_bn = (long long)d.ns * B * n * F;   // gqx, gqy
    const long long total = 2 * n_sn + 2 * n_bn;
    for (long long e = gtid(); e < total; e += gstride()) {
        float2 acc = make_float2(0.f, 0.f);
        if (e < 2 * n_sn) {
            const bool isx = e < n_sn;
            const long long r = isx ? e : e - n_sn;
            const int f = (int)(r % F);
            const int i = (int)((r / F) % n);
            const int s = (int)((r / ((long long)F * n)) % S);
            const int c = (int)(r / ((long long)F * n * S));
            const float2 a = d.params[d.a_off + f];
            for (int b = 0; b < B; ++b) {
                const long long cbs = ((long long)c * B + b) * S + s;
                const long long qi = (((long long)c * B + b) * n + i) * F + f;
                const float2 gv = (isx ? d.gXA : d.gY)[(cbs * n + i) * F + f];
                const float2 w = isx ? cmul(cmul(a, d.qx[qi]), d.qs[cbs * F + f]) : d.qy[qi];
                acc = cjmad(w, gv, acc);
            }
            (isx ? d.gXs : d.gYs)[r] = acc;
        } else if (e < 2 * n_sn + 2 * n_bn) {
            const long long e2 = e - 2 * n_sn;
            const bool isx = e2 < n_bn;
            const long long r = isx ? e2 : e2 - n_bn;
            const int f = (int)(r % F);
            const int i = (int)((r / F) % n);
            const int b = (int)((r / ((long long)F * n)) % B);
            const int c = (int)(r / ((long long)F * n * B));
            const float2 a = d.params[d.a_off + f];
            for (int s = 0; s < S; ++s) {
                const long long cbs = ((long long)c * B + b) * S + s;
                const long long si = (((long long)c * S + s) * n + i) * F + f;
                const float2 gv = (isx ? d.gXA : d.gY)[(cbs * n + i) * F + f];
                const float2 w = isx ? cmul(cmul(a, d.Xs[si]), d.qs[cbs * F + f]) : d.Ys[si];
                acc = cjmad(w, gv, acc);
            }
            (isx ? d.gqx : d.gqy)[r] = acc;
        }
    }
}

// h[c][b][s][f] = sum_x conj(Xs qx) gXA and gqs = conj(a) h: a wave per output, lane l
// summing x = l, l + 64, ... in order, then the wave's 64 partial sums by a fixed
// butterfly (every lane ends with the same total)
__global__ __launch_bounds__(kThreads) void k_kp_chain_h(const KPDesc d) {
    const int n = d.n, S = d.S, B = d.B, F = d.F;
    const long long n_bs = (long long)d.ns * B * S * F;
    const int lane = threadIdx.x & 63;
    for (long long r = (long long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); r < n_bs;
         r += (long long)gridDim.x * (kThreads / 64)) {
        const int f = (int)(r % F);
        const long long cbs = r / F;
        const int s = (int)(cbs % S);
        const int b = (int)((cbs / S) % B);
        const int c = (int)(cbs / ((long long)S * B));
        float2 acc = make_float2(0.f, 0.f);
        for (int x = lane; x < n; x += 64) {
            const float2 w = cmul(d.Xs[(((long long)c * S + s) * n + x) * F + f],
                                  d.qx[(((long long)c * B + b) * n + x) * F + f]);
            acc = cjmad(w, d.gXA[(cbs * n + x) * F + f], acc);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            acc.x += __shfl_xor(acc.x, o);
            acc.y += __shfl_xor(acc.y, o);
        }
        if (lane == 0) {
            d.h[r] = acc;
            d.gqs[r] = cjmad(d.params[d.a_off + f], acc, make_float2(0.f, 0.f));
        }
    }
}

// ga[f] = sum_c sum_b sum_s conj(qs) h: one block per feature, strided partial sums then
// a tree in a fixed order
__global__ __launch_bounds__(kThreads) void k_kp_chain_a(const KPDesc d) {
    __shared__ float2 red[kThreads];
    const int f = blockIdx.x;
    float2 acc = make_float2(0.f, 0.f);
    const long long nbs = (long long)d.ns * d.B * d.S;
    for (long long cbs = threadIdx.x; cbs < nbs; cbs += kThreads) acc = cjmad(d.qs[cbs * d.F + f], d.h[cbs * d.F + f], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) d.ga[f] = red[0];
}

// Which grid holds flat element e, and its index within the grid (a: plane KP_PLANES).
__device__ __forceinline__ void locate(const KPDesc& d, long long e, int* c, int* pl, long long* idx) {
    if (e >= d.a_off) {
        *c = 0; *pl = KP_PLANES; *idx = e - d.a_off;
        return;
    }
    for (int cc = d.ns - 1; cc >= 0; --cc)
        for (int p = KP_PLANES - 1; p >= 0; --p)
            if (e >= d.off[cc][p]) {
                *c = cc; *pl = p; *idx = e - d.off[cc][p];
                return;
            }
    *c = 0; *pl = 0; *idx = e;
}

// Length of a grid's first and second axes (F is the third).
__device__ __forceinline__ void grid_dims(const KPDesc& d, int c, int pl, int* d0, int* d1) {
    const int R = d.R[c];
    switch (pl) {
        case KP_XY: *d0 = R; *d1 = R; break;
        case KP_XS: case KP_YS: *d0 = d.S; *d1 = R; break;
        case KP_XT: case KP_YT: *d0 = d.Rt; *d1 = R; break;
        default: *d0 = d.Rt; *d1 = d.S; break;
    }
}

// Grid regulariser gradient (Section 4.3 readings): Charbonnier TV along the grid's x, y
// and omega axes, squared second differences along t and Charbonnier sparsity of p - 1
// on the time grids.
__device__ float2 reg_grad(const KPDesc& d, int c, int pl, int i0, int i1, int f, const float2* p) {
    int d0, d1;
    grid_dims(d, c, pl, &d0, &d1);
    const long long s0 = (long long)d1 * d.F, s1 = d.F;  // strides of the two axes
    const float2 v = p[0];
    float2 g = make_float2(-0.f, -0.f);
    const bool time = pl == KP_XT || pl == KP_YT || pl == KP_ST;
    if (d.tv_w != 0.f) {
        float2 t = make_float2(-0.f, -0.f);
        if (!time) {  // axis 0 is x, y or omega for the static grids
            if (i0 > 0) t = cadd(t, charb_w(csub(v, p[-s0]), d.eps2));
            if (i0 + 1 < d0) t = csub(t, charb_w(csub(p[s0], v), d.eps2));
        }
        if (i1 > 0) t = cadd(t, charb_w(csub(v, p[-s1]), d.eps2));
        if (i1 + 1 < d1) t = csub(t, charb_w(csub(p[s1], v), d.eps2));
        g = cfma(d.tv_w, t, g);
    }
    if (time && d.smooth_w != 0.f) {
        // d2_m = p[m+1] - 2 p[m] + p[m-1], m in [1, d0 - 2]; p[k] appears in m = k-1, k, k+1
        float2 t = make_float2(-0.f, -0.f);
        for (int m = i0 - 1; m <= i0 + 1; ++m) {
            if (m < 1 || m > d0 - 2) continue;
            const float2* q = p + (long long)(m - i0) * s0;
            const float2 d2 = cadd(csub(q[s0], cscale(q[0], 2.f)), q[-s0]);
            const float coef = m == i0 ? -4.f : 2.f;
            t = cfma(coef, d2, t);
        }
        g = cfma(d.smooth_w, t, g);
    }
    if (time && d.sparse_w != 0.f) g = cfma(d.sparse_w, charb_w(make_float2(v.x - 1.f, v.y), d.eps2), g);
    return g;
}

// Data gradient of every grid element (transposed interpolation, gather form) plus the
// regulariser gradient -> grad.
__global__ __launch_bounds__(kThreads) void k_kp_grid(const KPDesc d) {
    const int n = d.n, S = d.S, F = d.F;
    for (long long e = gtid(); e < d.n_params; e += gstride()) {
        int c, pl;
        long long idx;
        locate(d, e, &c, &pl, &idx);
        if (pl == KP_PLANES) {
            d.grad[e] = d.ga[idx];
            continue;
        }
        int d0, d1;
        grid_dims(d, c, pl, &d0, &d1);
        const int f = (int)(idx % F);
        const int i1 = (int)((idx / F) % d1);
        const int i0 = (int)(idx / ((long long)F * d1));
        const int* tp = d.tr_ptr + c * (n + 1);
        float2 acc = make_float2(0.f, 0.f);
        switch (pl) {
            case KP_XY:  // rows i0 (y nodes), columns i1 (x nodes)
                for (int a = tp[i0]; a < tp[i0 + 1]; ++a) {
                    const int y = d.tr_smp[a];
                    float2 row = make_float2(0.f, 0.f);
                    for (int q = tp[i1]; q < tp[i1 + 1]; ++q)
                        row = cfma(d.tr_w[q], d.gZ[(((long long)c * n + y) * n + d.tr_smp[q]) * F + f], row);
                    acc = cfma(d.tr_w[a], row, acc);
                }
                break;
            case KP_XS:
            case KP_YS: {
                const float2* src = pl == KP_XS ? d.gXs : d.gYs;
                for (int q = tp[i1]; q < tp[i1 + 1]; ++q)
                    acc = cfma(d.tr_w[q], src[(((long long)c * S + i0) * n + d.tr_smp[q]) * F + f], acc);
                break;
            }
            case KP_XT:
            case KP_YT: {
                const float2* src = pl == KP_XT ? d.gqx : d.gqy;
                for (int t = d.tt_ptr[i0]; t < d.tt_ptr[i0 + 1]; ++t) {
                    const int b = d.tt_b[t];
                    float2 part = make_float2(0.f, 0.f);
                    for (int q = tp[i1]; q < tp[i1 + 1]; ++q)
                        part = cfma(d.tr_w[q], src[(((long long)c * d.B + b) * n + d.tr_smp[q]) * F + f], part);
                    acc = cfma(d.tt_w[t], part, acc);
                }
                break;
            }
            default:  // omega-t: rows i0 (time nodes), columns i1 (bins)
                for (int t = d.tt_ptr[i0]; t < d.tt_ptr[i0 + 1]; ++t)
                    acc = cfma(d.tt_w[t], d.gqs[(((long long)c * d.B + d.tt_b[t]) * S + i1) * F + f], acc);
                break;
        }
        d.grad[e] = cadd(acc, reg_grad(d, c, pl, i0, i1, f, d.params + e));
    }
}

// Regulariser value: per element its forward differences (TV), the second difference
// centred on it (smoothness) and its sparsity term, as |z|^2 / (sqrt(|z|^2 + e^2) + e) for
// the Charbonnier terms; FP64 block sums in a fixed order -> rpart[block].
__global__ __launch_bounds__(kThreads) void k_kp_reg_value(const KPDesc d) {
    __shared__ double red[kThreads];
    const double e2 = (double)d.eps2, ep = sqrt(e2);
    auto charb = [&](float2 z) {
        const double q = (double)z.x * z.x + (double)z.y * z.y;
        return q / (sqrt(q + e2) + ep);
    };
    double acc = 0.0;
    for (long long e = gtid(); e < d.a_off; e += gstride()) {
        int c, pl;
        long long idx;
        locate(d, e, &c, &pl, &idx);
        int d0, d1;
        grid_dims(d, c, pl, &d0, &d1);
        const int i1 = (int)((idx / d.F) % d1);
        const int i0 = (int)(idx / ((long long)d.F * d1));
        const long long s0 = (long long)d1 * d.F, s1 = d.F;
        const float2* p = d.params + e;
        const bool time = pl == KP_XT || pl == KP_YT || pl == KP_ST;
        if (d.tv_w != 0.f) {
            double t = 0.0;
            if (!time && i0 + 1 < d0) t += charb(csub(p[s0], p[0]));
            if (i1 + 1 < d1) t += charb(csub(p[s1], p[0]));
            acc += (double)d.tv_w * t;
        }
        if (time && d.smooth_w != 0.f && i0 >= 1 && i0 <= d0 - 2) {
            const double rx = ((double)p[s0].x - 2.0 * p[0].x) + p[-s0].x;
            const double ry = ((double)p[s0].y - 2.0 * p[0].y) + p[-s0].y;
            acc += (double)d.smooth_w * (rx * rx + ry * ry);
        }
        if (time && d.sparse_w != 0.f) acc += (double)d.sparse_w * charb(make_float2(p[0].x - 1.f, p[0].y));
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.rpart[blockIdx.x] = red[0];
}

// Adam (or GD) on every parameter, (Re, Im) as independent reals; step t = counter + 1.
__global__ __launch_bounds__(kThreads) void k_kp_update(const KPDesc d) {
    const int st = d.step ? *d.step : 0;
    const bool adam = d.optimizer == VP_OPT_ADAM;
    float step_size = d.lr, inv_bc2s = 1.f;
    if (adam) {
        const float tf = (float)(st + 1);
        const float bc1 = -expm1f(tf * d.ln_beta1), bc2 = -expm1f(tf * d.ln_beta2);
        step_size = d.lr / bc1;
        inv_bc2s = 1.f / sqrtf(bc2);
    }
    float2* p = const_cast<float2*>(d.params);
    for (long long e = gtid(); e < d.n_params; e += gstride()) {
        const float2 g = d.grad[e], v0 = p[e];
        if (adam) {
            float2 m = d.m[e], v = d.v[e];
            m.x = __builtin_fmaf(d.beta1, m.x, d.c1 * g.x);
            m.y = __builtin_fmaf(d.beta1, m.y, d.c1 * g.y);
            v.x = __builtin_fmaf(d.beta2, v.x, (d.c2 * g.x) * g.x);
            v.y = __builtin_fmaf(d.beta2, v.y, (d.c2 * g.y) * g.y);
            d.m[e] = m;
            d.v[e] = v;
            const float dx = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.x), inv_bc2s, d.aeps);
            const float dy = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.y), inv_bc2s, d.aeps);
            p[e] = make_float2(__builtin_fmaf(-step_size, m.x * __builtin_amdgcn_rcpf(dx), v0.x),
                               __builtin_fmaf(-step_size, m.y * __builtin_amdgcn_rcpf(dy), v0.y));
        } else {
            p[e] = make_float2(__builtin_fmaf(-d.lr, g.x, v0.x), __builtin_fmaf(-d.lr, g.y, v0.y));
        }
    }
}

__global__ void k_kp_advance(int* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step = *step + 1;
}

// proj / water / fat of vol [B][S][n][n]
__global__ __launch_bounds__(kThreads) void k_kp_render(const KPDesc d, int split, float2* proj, float2* water,
                                                        float2* fat) {
    const long long nn = (long long)d.n * d.n;
    const long long total = (long long)d.B * nn;
    for (long long e = gtid(); e < total; e += gstride()) {
        const long long b = e / nn, px = e % nn;
        float2 w = make_float2(0.f, 0.f), ft = w;
        for (int s = 0; s < d.S; ++s) {
            const float2 v = d.vol[(b * d.S + s) * nn + px];
            if (s < split) w = cadd(w, v);
            else ft = cadd(ft, v);
        }
        if (proj) proj[e] = cadd(w, ft);
        if (water) water[e] = w;
        if (fat) fat[e] = ft;
    }
}

inline unsigned grid_of(long long total) {
    const long long g = (total + kThreads - 1) / kThreads;
    return (unsigned)(g < 1 ? 1 : (g > (1 << 20) ? (1 << 20) : g));
}

}  // namespace

bool kp_features_ok(int f) { return f == 1 || f == 2 || f == 4 || f == 8 || f == 16; }

hipError_t kp_launch_factors(const KPDesc& d, hipStream_t s) {
    const dim3 b(kThreads);
    hipLaunchKernelGGL(k_kp_fac_s, dim3(grid_of((long long)d.ns * d.S * d.n * d.F)), b, 0, s, d);
    hipLaunchKernelGGL(k_kp_fac_t, dim3(grid_of((long long)d.ns * d.B * (d.n + d.S) * d.F)), b, 0, s, d);
    hipLaunchKernelGGL(k_kp_fac_z, dim3(grid_of((long long)d.ns * d.n * d.n * d.F)), b, 0, s, d);
    hipLaunchKernelGGL(k_kp_prod, dim3(grid_of((long long)d.ns * d.B * d.S * d.n * d.F)), b, 0, s, d);
    return hipGetLastError();
}

#define KP_F_SWITCH(KERNEL, GRID)                                                   \
    switch (d.F) {                                                                  \
        case 1: hipLaunchKernelGGL(KERNEL<1>, GRID, dim3(kThreads), 0, s, d); break;   \
        case 2: hipLaunchKernelGGL(KERNEL<2>, GRID, dim3(kThreads), 0, s, d); break;   \
        case 4: hipLaunchKernelGGL(KERNEL<4>, GRID, dim3(kThreads), 0, s, d); break;   \
        case 8: hipLaunchKernelGGL(KERNEL<8>, GRID, dim3(kThreads), 0, s, d); break;   \
        case 16: hipLaunchKernelGGL(KERNEL<16>, GRID, dim3(kThreads), 0, s, d); break; \
        default: return hipErrorInvalidValue;                                       \
    }

hipError_t kp_launch_decode(const KPDesc& d, hipStream_t s) {
    KP_F_SWITCH(k_kp_decode, dim3(grid_of((long long)d.B * ((d.S + kDecBins - 1) / kDecBins) * ((d.n + kDecRows - 1) / kDecRows) * ((d.n + 63) / 64) * 64)));
    return hipGetLastError();
}

hipError_t kp_launch_back_z(const KPDesc& d, hipStream_t s) {
    KP_F_SWITCH(k_kp_grad_z, dim3(grid_of((long long)d.zchunks * ((d.n + kGzRows - 1) / kGzRows) * ((d.n + 63) / 64) * 64)));
    hipLaunchKernelGGL(k_kp_grad_z_sum, dim3(grid_of((long long)d.ns * d.n * d.n * d.F)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t kp_launch_back_x(const KPDesc& d, hipStream_t s) {
    KP_F_SWITCH(k_kp_grad_x, dim3(grid_of((long long)((d.B * d.S + kGxBs - 1) / kGxBs) * ((d.n + 63) / 64) * 64 * kGxYs)));
    hipLaunchKernelGGL(k_kp_gx_sum, dim3(grid_of((long long)d.ns * d.B * d.S * d.n * d.F)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}
hipError_t kp_launch_back_y(const KPDesc& d, hipStream_t s) {
    // as the kernel's blocks of RB (b, s) by RY rows, RB RY = 32 / F
    const int rw = 32 / d.F, ry = rw >= 16 ? 4 : (rw >= 4 ? 2 : 1), rb = rw / ry;
    const long long groups = ((long long)(d.B * d.S + rb - 1) / rb) * ((d.n + ry - 1) / ry);
    const long long blocks = (groups + kThreads / 64 - 1) / (kThreads / 64);
    KP_F_SWITCH(k_kp_grad_y, dim3((unsigned)(blocks > (1 << 20) ? (1 << 20) : blocks)));
    return hipGetLastError();
}
hipError_t kp_launch_back(const KPDesc& d, hipStream_t s) {
    hipError_t e = kp_launch_back_z(d, s);
    if (e == hipSuccess) e = kp_launch_back_x(d, s);
    if (e == hipSuccess) e = kp_launch_back_y(d, s);
    return e;
}
#undef KP_F_SWITCH

hipError_t kp_launch_chain(const KPDesc& d, hipStream_t s) {
    const long long total = 2LL * d.ns * d.S * d.n * d.F + 2LL * d.ns * d.B * d.n * d.F;
    hipLaunchKernelGGL(k_kp_chain1, dim3(grid_of(total)), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_kp_chain_h, dim3(grid_of((long long)d.ns * d.B * d.S * d.F * 64)), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_kp_chain_a, dim3(d.F), dim3(kThreads), 0, s, d);
    hipLaunchKernelGGL(k_kp_grid, dim3(grid_of(d.n_params)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}

hipError_t kp_launch_update(const KPDesc& d, hipStream_t s) {
    hipLaunchKernelGGL(k_kp_update, dim3(grid_of(d.n_params)), dim3(kThreads), 0, s, d);
    if (d.step) hipLaunchKernelGGL(k_kp_advance, dim3(1), dim3(64), 0, s, d.step);
    return hipGetLastError();
}

int kp_reg_blocks(const KPDesc& d) {
    const long long g = (d.a_off + kThreads - 1) / kThreads;
    return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

hipError_t kp_launch_reg_value(const KPDesc& d, hipStream_t s) {
    hipLaunchKernelGGL(k_kp_reg_value, dim3(kp_reg_blocks(d)), dim3(kThreads), 0, s, d);
    return hipGetLastError();
}

hipError_t kp_launch_render(const KPDesc& d, int split, float2* proj, float2* water, float2* fat, hipStream_t s) {
    hipLaunchKernelGGL(k_kp_render, dim3(grid_of((long long)d.B * d.n * d.n)), dim3(kThreads), 0, s, d, split, proj,
                       water, fat);
    return hipGetLastError();
}

}  // namespace vp
