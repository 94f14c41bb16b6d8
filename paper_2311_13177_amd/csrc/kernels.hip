// HIP kernels (gfx950) of the lifted-PROPELLER hot path.
//
// Every kernel walks a list of work items (Task) with a grid-stride loop, so one
// launch can cover one slice or many slices of different sizes; each item reads its
// slice descriptor. Per-voxel and per-pixel summation orders depend only on the
// slice's own plan (bins ascending, blade parts in plan order, fixed tap order), never
// on the batch, the tile or the wave that happens to hold the element.
//
// Stages of one optimiser step (Sections 4.2 and 4.3 of the paper):
//   k_project   sheared spectral projection of a knot's volume for a group of blade
//               parts; the bin plane is staged in LDS once per block and shared by
//               the four waves, each accumulating its own parts
//   k_rows<FWD> blend of a blade's knot projections, forward DFT of every row
//   k_cols      forward DFT of every column, 1/n scaling, blade mask, residual
//               against the measurement, loss partials, inverse DFT of the column
//   k_rows<INV> inverse DFT of every row: the image-space residual g_b
//   k_gather    transposed shear as a gather over blade parts (no atomics); each
//               blade image region is staged in LDS once per block and the four waves
//               accumulate disjoint bins; fused epilogue: TV/L1 gradient and the Adam
//               or GD update, and the step counter advanced by the last work item
//
// Uniform data (work items, descriptors, shear table, blade and knot tables) is read
// through constant-address-space pointers so that it lands in scalar registers.

#include <hip/hip_runtime.h>

#include "vp.h"
#include "vp_internal.h"

namespace vp {

#define AS4 __attribute__((address_space(4)))

template <class T>
__device__ __forceinline__ const AS4 T* cst(const T* p) {
    return (const AS4 T*)(const void*)p;
}

// Field of the work item's slice descriptor (descriptor array or the inline copy).
#define DF(field) (a.descs ? cst(a.descs + slice)->field : a.one.field)

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// (sign * i) * a
template <int SIGN>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// acc + w * a, one fused multiply-add per component
__device__ __forceinline__ float2 cfma(float w, float2 a, float2 acc) {
    return make_float2(__builtin_fmaf(w, a.x, acc.x), __builtin_fmaf(w, a.y, acc.y));
}
__device__ __forceinline__ bool active_blade(int sched, const int* stepp, int st, int B, int b) {
    return sched != VP_SCHED_CYCLIC || stepp == nullptr || b == st % B;
}
__device__ __forceinline__ int read_step(const int* stepp) { return stepp ? *cst(stepp) : 0; }

// ------------------------------------------------------------------ DFT in LDS
//
// Mixed-radix Stockham autosort (radices 2, 3, 4, 5), in place: in every stage each
// thread reads the inputs of its butterflies into registers, the block synchronises,
// and each thread writes its outputs. `count` transforms of length n live in LDS:
// element j of transform f at buf[f * fstride + j * estride], with n * count <= E *
// kThreads. Twiddles exp(-2 pi i j / n) are read from an LDS table. DIR = -1 is the
// forward transform, DIR = +1 the unnormalised inverse. The stage radices come packed
// three bits per stage.

template <int DIR, int R>
__device__ __forceinline__ void butterfly(float2 (&x)[R]) {
    if constexpr (R == 2) {
        const float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (R == 4) {
        const float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
        const float2 t2 = cadd(x[1], x[3]), t3 = mul_i<DIR>(csub(x[1], x[3]));
        x[0] = cadd(t0, t2);
        x[1] = cadd(t1, t3);
        x[2] = csub(t0, t2);
        x[3] = csub(t1, t3);
    } else if constexpr (R == 3) {
        const float s3 = 0.86602540378443864676f;  // sin(2 pi / 3)
        const float2 t = cadd(x[1], x[2]);
        const float2 u = mul_i<DIR>(cscale(csub(x[1], x[2]), s3));
        const float2 h = make_float2(x[0].x - 0.5f * t.x, x[0].y - 0.5f * t.y);
        x[0] = cadd(x[0], t);
        x[1] = cadd(h, u);
        x[2] = csub(h, u);
    } else if constexpr (R == 5) {
        const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
        const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
        const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
        const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
        const float2 a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
        const float2 a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
        const float2 x0 = x[0];
        const float2 p1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        const float2 p2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        const float2 q1 = mul_i<DIR>(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        const float2 q2 = mul_i<DIR>(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        x[0] = cadd(x0, cadd(a1, a2));
        x[1] = cadd(p1, q1);
        x[2] = cadd(p2, q2);
        x[3] = csub(p2, q2);
        x[4] = csub(p1, q1);
    }
}

template <int DIR, int R, bool FFAST, int E>
__device__ __forceinline__ void stockham_stage(float2* buf, const float2* tw, int n, int count, int fstride,
                                               int estride, int p) {
    constexpr int MAXB = (E + R - 1) / R;  // butterflies per thread (n * count <= E * kThreads)
    const int m = n / R;
    const int total = m * count;
    const int tws = n / (p * R);
    float2 x[MAXB][R];
    int bout[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        bout[t] = -1;
        if (idx < total) {
            int f, j;
            if (FFAST) {
                f = idx % count;
                j = idx / count;
            } else {
                j = idx % m;
                f = idx / m;
            }
            const int k = j % p;
            const int bin = f * fstride + j * estride;
            bout[t] = f * fstride + ((j - k) * R + k) * estride;
#pragma unroll
            for (int q = 0; q < R; ++q) x[t][q] = buf[bin + q * m * estride];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                float2 w = tw[k * q * tws];
                if (DIR > 0) w.y = -w.y;
                x[t][q] = cmul(x[t][q], w);
            }
            butterfly<DIR, R>(x[t]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        if (bout[t] >= 0) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[bout[t] + q * p * estride] = x[t][q];
        }
    }
    __syncthreads();
}

template <int DIR, bool FFAST, int E>
__device__ void lds_fft(float2* buf, const float2* tw, int n, int count, int fstride, int estride, int nstage,
                        int code) {
    int p = 1;
    for (int st = 0; st < nstage; ++st) {
        const int r = (code >> (3 * st)) & 7;
        switch (r) {
            case 4: stockham_stage<DIR, 4, FFAST, E>(buf, tw, n, count, fstride, estride, p); break;
            case 2: stockham_stage<DIR, 2, FFAST, E>(buf, tw, n, count, fstride, estride, p); break;
            case 3: stockham_stage<DIR, 3, FFAST, E>(buf, tw, n, count, fstride, estride, p); break;
            default: stockham_stage<DIR, 5, FFAST, E>(buf, tw, n, count, fstride, estride, p); break;
        }
        p *= r;
    }
}

// Compile-time variant for the common lengths: the radix sequence, strides and index
// arithmetic are constants (the same factorisation as the plan: 4s, then 2s, 3s, 5s,
// so results equal the runtime variant's bit for bit).
__host__ __device__ constexpr int ct_radix(int n, int i) {
    int st = 0;
    while (n % 4 == 0) { if (st == i) return 4; n /= 4; ++st; }
    while (n % 2 == 0) { if (st == i) return 2; n /= 2; ++st; }
    while (n % 3 == 0) { if (st == i) return 3; n /= 3; ++st; }
    while (n % 5 == 0) { if (st == i) return 5; n /= 5; ++st; }
    return 0;
}

template <int DIR, int R, bool FFAST, int N, int COUNT, int P>
__device__ __forceinline__ void ct_stage(float2* buf, const float2* tw) {
    constexpr int m = N / R, total = m * COUNT, tws = N / (P * R);
    constexpr int FS = FFAST ? 1 : N, ES = FFAST ? COUNT : 1;
    constexpr int MAXB = (total + kThreads - 1) / kThreads;
    float2 x[MAXB][R];
    int bout[MAXB];
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        const int idx = threadIdx.x + t * kThreads;
        bout[t] = -1;
        if (total % kThreads == 0 || idx < total) {
            const int f = FFAST ? idx % COUNT : idx / m;
            const int j = FFAST ? idx / COUNT : idx % m;
            const int k = j % P;
            const int bin = f * FS + j * ES;
            bout[t] = f * FS + ((j - k) * R + k) * ES;
#pragma unroll
            for (int q = 0; q < R; ++q) x[t][q] = buf[bin + q * m * ES];
#pragma unroll
            for (int q = 1; q < R; ++q) {
                float2 w = tw[k * q * tws];
                if (DIR > 0) w.y = -w.y;
                x[t][q] = cmul(x[t][q], w);
            }
            butterfly<DIR, R>(x[t]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < MAXB; ++t) {
        if (bout[t] >= 0) {
#pragma unroll
            for (int q = 0; q < R; ++q) buf[bout[t] + q * P * ES] = x[t][q];
        }
    }
    __syncthreads();
}

template <int DIR, bool FFAST, int N, int COUNT, int ST = 0, int P = 1>
__device__ __forceinline__ void ct_fft(float2* buf, const float2* tw) {
    if constexpr (ct_radix(N, ST) != 0) {
        constexpr int R = ct_radix(N, ST);
        ct_stage<DIR, R, FFAST, N, COUNT, P>(buf, tw);
        ct_fft<DIR, FFAST, N, COUNT, ST + 1, P * R>(buf, tw);
    }
}

// Row transforms (count rows of length n, row-major) and column transforms (count
// columns of length n, element j of column f at j * count + f), dispatched to the
// compile-time variant for the common lengths.
template <int DIR>
__device__ void fft_rows_any(float2* buf, const float2* tw, int n, int nstage, int code) {
    switch (n) {
        case 64: ct_fft<DIR, false, 64, fft_rows_per_item(64)>(buf, tw); break;
        case 128: ct_fft<DIR, false, 128, fft_rows_per_item(128)>(buf, tw); break;
        case 192: ct_fft<DIR, false, 192, fft_rows_per_item(192)>(buf, tw); break;
        case 256: ct_fft<DIR, false, 256, fft_rows_per_item(256)>(buf, tw); break;
        case 320: ct_fft<DIR, false, 320, fft_rows_per_item(320)>(buf, tw); break;
        case 384: ct_fft<DIR, false, 384, fft_rows_per_item(384)>(buf, tw); break;
        default: lds_fft<DIR, false, 8>(buf, tw, n, fft_rows_per_item(n), n, 1, nstage, code); break;
    }
}
template <int DIR>
__device__ void fft_cols_any(float2* buf, const float2* tw, int n, int nstage, int code) {
    switch (n) {
        case 64: ct_fft<DIR, true, 64, fft_cols_per_item(64)>(buf, tw); break;
        case 128: ct_fft<DIR, true, 128, fft_cols_per_item(128)>(buf, tw); break;
        case 192: ct_fft<DIR, true, 192, fft_cols_per_item(192)>(buf, tw); break;
        case 256: ct_fft<DIR, true, 256, fft_cols_per_item(256)>(buf, tw); break;
        case 320: ct_fft<DIR, true, 320, fft_cols_per_item(320)>(buf, tw); break;
        case 384: ct_fft<DIR, true, 384, fft_cols_per_item(384)>(buf, tw); break;
        default: {
            const int cb = fft_cols_per_item(n);
            lds_fft<DIR, true, 16>(buf, tw, n, cb, 1, cb, nstage, code);
            break;
        }
    }
}

// ------------------------------------------------------------------ LDS staging
//
// A rectangular region (rows x cols) of an n x n image, origin (gy0, gx0), is staged
// into LDS with zeros outside the image. Each thread owns region elements
// threadIdx.x + k * kThreads (k < SE); their image offsets are computed once per work
// item, and the next plane's values are loaded into registers while the current plane
// is being consumed (double-buffered LDS, one barrier per plane).

// P planes (images of the same size, same region) are staged per phase; plane p of a
// phase occupies buf[p * re, (p + 1) * re). A null plane pointer stages zeros.
template <int SE, int P>
struct Stager {
    int off[SE];
    int re;
    __device__ void init(int rows, int cols, int gy0, int gx0, int n) {
        re = rows * cols;
#pragma unroll
        for (int k = 0; k < SE; ++k) {
            const int i = threadIdx.x + k * kThreads;
            int o = -1;
            if (i < re) {
                const int r = i / cols, c = i - (i / cols) * cols;
                const int gy = gy0 + r, gx = gx0 + c;
                if (gy >= 0 && gy < n && gx >= 0 && gx < n) o = gy * n + gx;
            }
            off[k] = i < re ? o : -2;
        }
    }
    __device__ void fetch(const float2* const (&img)[P], float2 (&pre)[P][SE]) const {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < SE; ++k) {
                float2 v = make_float2(0.f, 0.f);
                if (img[p] && off[k] >= 0) v = img[p][off[k]];
                pre[p][k] = v;
            }
    }
    __device__ void store(float2* buf, const float2 (&pre)[P][SE]) const {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < SE; ++k)
                if (off[k] != -2) buf[p * re + threadIdx.x + k * kThreads] = pre[p][k];
    }
};

// ------------------------------------------------------------------ projection
//
// P_b[y][x] = sum_s sum_taps w * V_s[y + oy + (0|1)][x + ox + (0|1)]   (Section 4.2)
// Work item: (part group, tile row, tile column), tile = 64 columns x kTileRows rows.
// Part e of the group belongs to wave e % 4, slot e / 4. Each lane owns one column.

template <int GW, int SE, int P>
__global__ __launch_bounds__(kThreads) void k_project(const KArgs a) {
    extern __shared__ float2 sm[];
    constexpr int PPT = kTileRows;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S), B = DF(B), nparts = DF(nparts), sched = DF(schedule);
        const size_t nn = (size_t)n * n;
        const AS4 ProjGroup* gr = cst(DF(groups)) + tk->a;
        const int knot = gr->knot, ge0 = gr->e0, gne = gr->ne;
        const int oxmin = gr->ox_min, oymin = gr->oy_min;
        const int RH = PPT + gr->oy_max - oymin + 1, RW = kTileW + gr->ox_max - oxmin + 1;
        const int RE = RH * RW;
        const int y0 = tk->b * PPT, x0 = tk->c * kTileW;
        const AS4 KnotEntry* ent = cst(DF(knot_ent));
        const AS4 ShearEntry* shear = cst(DF(shear));
        float2* const work = DF(work);
        const float2* const V = (stepp ? DF(vol[st & 1]) : DF(vol[0])) + (size_t)knot * S * nn;
        int eb[GW], ep[GW];
        bool act[GW];
#pragma unroll
        for (int j = 0; j < GW; ++j) {
            const int e = j * 4 + wave;
            act[j] = false;
            eb[j] = 0;
            ep[j] = 0;
            if (e < gne) {
                eb[j] = ent[ge0 + e].blade;
                ep[j] = ent[ge0 + e].part;
                act[j] = active_blade(sched, stepp, st, B, eb[j]);
            }
        }
        float2 acc[GW][PPT];
#pragma unroll
        for (int j = 0; j < GW; ++j)
#pragma unroll
            for (int i = 0; i < PPT; ++i) acc[j][i] = make_float2(0.f, 0.f);
        Stager<SE, P> sg;
        sg.init(RH, RW, y0 + oymin, x0 + oxmin, n);
        float2 pre[P][SE];
        {
            const float2* planes[P];
#pragma unroll
            for (int p = 0; p < P; ++p) planes[p] = p < S ? V + (size_t)p * nn : nullptr;
            sg.fetch(planes, pre);
        }
        for (int s0 = 0, it = 0; s0 < S; s0 += P, ++it) {
            float2* buf = sm + (it & 1) * P * RE;
            sg.store(buf, pre);
            __syncthreads();
            if (s0 + P < S) {
                const float2* planes[P];
#pragma unroll
                for (int p = 0; p < P; ++p) planes[p] = s0 + P + p < S ? V + (size_t)(s0 + P + p) * nn : nullptr;
                sg.fetch(planes, pre);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int s = s0 + p;
                if (s < S) {
#pragma unroll
                    for (int j = 0; j < GW; ++j) {
                        if (act[j]) {
                            const AS4 ShearEntry* sh = shear + eb[j] * S + s;
                            const float w00 = sh->w00, w01 = sh->w01, w10 = sh->w10, w11 = sh->w11;
                            const float2* L = buf + p * RE + (sh->oy - oymin) * RW + (sh->ox - oxmin) + lane;
                            float2 a0 = L[0], a1 = L[1];
#pragma unroll
                            for (int i = 0; i < PPT; ++i) {
                                const float2 b0 = L[(i + 1) * RW], b1 = L[(i + 1) * RW + 1];
                                float2 t = acc[j][i];
                                t = cfma(w00, a0, t);
                                t = cfma(w01, a1, t);
                                t = cfma(w10, b0, t);
                                t = cfma(w11, b1, t);
                                acc[j][i] = t;
                                a0 = b0;
                                a1 = b1;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
        const int x = x0 + lane;
#pragma unroll
        for (int j = 0; j < GW; ++j) {
            if (act[j] && x < n) {
                float2* out = work + ((size_t)eb[j] * nparts + ep[j]) * nn;
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    const int y = y0 + i;
                    if (y < n) out[(size_t)y * n + x] = acc[j][i];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ row passes
//
// DIR = -1: blend the blade's knot projections, (1 - a) P_k + a P_{k+1}, and take the
// forward DFT of each row. DIR = +1: inverse DFT of each row (the column pass has
// already applied both unitary scalings).

template <int DIR>
__global__ __launch_bounds__(kThreads) void k_rows(const KArgs a) {
    extern __shared__ float2 sm[];
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int b = tk->a;
        if (!active_blade(DF(schedule), stepp, st, DF(B), b)) continue;
        const int n = DF(n), nparts = DF(nparts), nstage = DF(nstage), code = DF(radix_code);
        const size_t nn = (size_t)n * n;
        const int fb = fft_rows_per_item(n);
        const int r0 = tk->b, rows = min(fb, n - r0);
        float2* A = sm;
        float2* tw = sm + fb * n;
        float2* img = DF(work) + (size_t)b * nparts * nn;
        const float2* twg = DF(tw);
        const size_t base = (size_t)r0 * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
        if (DIR < 0 && nparts == 2) {
            const AS4 BladeDev* bd = cst(DF(blade)) + b;
            const int has0 = bd->has0, has1 = bd->has1;
            const float w0 = bd->w0, w1 = bd->w1;
            const float2* p1 = img + nn;
            for (int i = threadIdx.x; i < fb * n; i += blockDim.x) {
                float2 v = make_float2(0.f, 0.f);
                if (i < rows * n) {
                    if (has0) v = cscale(img[base + i], w0);
                    if (has1) v = cfma(w1, p1[base + i], v);
                }
                A[i] = v;
            }
        } else {
            for (int i = threadIdx.x; i < fb * n; i += blockDim.x)
                A[i] = i < rows * n ? img[base + i] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        fft_rows_any<DIR>(A, tw, n, nstage, code);
        for (int i = threadIdx.x; i < rows * n; i += blockDim.x) img[base + i] = A[i];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ column pass
//
// COL_STEP:    forward column DFT, K = X / n, R = M (K - y), loss partial sum |R|^2,
//              Z = R / n, inverse column DFT -> work (one pass per column strip).
// COL_FORWARD: forward column DFT, out = M (K - y) (y optional), no inverse.
// COL_ADJOINT: reads caller k-space, Z = M kres / n, inverse column DFT -> work.

__global__ __launch_bounds__(kThreads) void k_cols(const KArgs a) {
    extern __shared__ float2 sm[];
    __shared__ float red[kThreads];
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int b = tk->a;
        float* const loss_part = DF(loss_part);
        const int n_col_items = DF(n_col_items);
        if (!active_blade(DF(schedule), stepp, st, DF(B), b)) {
            if (a.mode == COL_STEP && threadIdx.x == 0) loss_part[b * n_col_items + tk->b] = 0.f;
            continue;
        }
        const int n = DF(n), nparts = DF(nparts), nstage = DF(nstage), code = DF(radix_code);
        const size_t nn = (size_t)n * n;
        const int cb = fft_cols_per_item(n);
        const int c0 = tk->b * cb, cols = min(cb, n - c0);
        float2* A = sm;
        float2* tw = sm + cb * n;
        float2* img = DF(work) + (size_t)b * nparts * nn;
        const float2* twg = DF(tw);
        const float2* src = a.mode == COL_ADJOINT ? a.in0 + (size_t)b * nn : img;
        for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
        for (int i = threadIdx.x; i < n * cb; i += blockDim.x) {
            const int y = i / cb, c = i - (i / cb) * cb;
            A[i] = c < cols ? src[(size_t)y * n + c0 + c] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        if (a.mode != COL_ADJOINT) fft_cols_any<-1>(A, tw, n, nstage, code);
        const float sc = 1.0f / (float)n;
        const uint8_t* mk = DF(mask) + (size_t)b * nn;
        const float2* yy = DF(y);
        const float2* yb = yy ? yy + (size_t)b * nn : nullptr;
        float lsum = 0.f;
        for (int i = threadIdx.x; i < n * cb; i += blockDim.x) {
            const int y = i / cb, c = i - (i / cb) * cb;
            float2 v = make_float2(0.f, 0.f);
            if (c < cols) {
                const size_t gi = (size_t)y * n + c0 + c;
                const bool on = mk[gi] != 0;
                const float2 x = A[i];
                if (a.mode == COL_ADJOINT) {
                    if (on) v = cscale(x, sc);
                } else {
                    float2 r = make_float2(0.f, 0.f);
                    if (on) {
                        r = cscale(x, sc);
                        if (yb) r = csub(r, yb[gi]);
                    }
                    if (a.mode == COL_FORWARD) {
                        a.out0[(size_t)b * nn + gi] = r;
                    } else {
                        lsum = __builtin_fmaf(r.x, r.x, lsum);
                        lsum = __builtin_fmaf(r.y, r.y, lsum);
                        v = cscale(r, sc);
                    }
                }
            }
            A[i] = v;
        }
        __syncthreads();
        if (a.mode != COL_FORWARD) {
            fft_cols_any<1>(A, tw, n, nstage, code);
            for (int i = threadIdx.x; i < n * cb; i += blockDim.x) {
                const int y = i / cb, c = i - (i / cb) * cb;
                if (c < cols) img[(size_t)y * n + c0 + c] = A[i];
            }
        }
        if (a.mode == COL_STEP) {
            red[threadIdx.x] = lsum;
            __syncthreads();
            for (int w = kThreads / 2; w > 0; w >>= 1) {
                if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
                __syncthreads();
            }
            if (threadIdx.x == 0) loss_part[b * n_col_items + tk->b] = red[0];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ regulariser gradient

// Charbonnier weight d / sqrt(|d|^2 + eps^2): the gradient of sqrt(|d|^2 + eps^2) - eps.
__device__ __forceinline__ float2 charb_w(float2 dlt, float eps2) {
    return cscale(dlt, rsqrtf(dlt.x * dlt.x + dlt.y * dlt.y + eps2));
}

// tv_w * grad TV + l1_w * grad L1 at voxel (t, s, y, x) of a [T][S][n][n] volume.
__device__ __forceinline__ float2 reg_grad(const float2* __restrict__ V, size_t idx, int t, int s, int y, int x,
                                           int n, int S, int T, float tv_w, float l1_w, float eps) {
    const float eps2 = eps * eps;
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

__device__ __forceinline__ float2 shfl_up1(float2 v) { return make_float2(__shfl_up(v.x, 1), __shfl_up(v.y, 1)); }
__device__ __forceinline__ float2 shfl_down1(float2 v) {
    return make_float2(__shfl_down(v.x, 1), __shfl_down(v.y, 1));
}

// ------------------------------------------------------------------ optimiser update of a column

struct UpdateArgs {
    int n, S, T, kt, y0, x0, lane, sw, ns, opt;
    float lr, beta1, beta2, aeps, tv_w, l1_w, eps2, inv_bc2s, step_size;
};

// Adds the TV/L1 gradient to the data gradient acc of one lane's voxels (bins sw ..
// sw + ns - 1, rows y0 .. y0 + PPT - 1, column x0 + lane of knot kt) and applies Adam
// or GD, reading Vin and writing Vout (distinct buffers, as are the moments). The lane
// walks its bins with a register window of the previous, current and next bin (rows
// y0 - 1 .. y0 + PPT, zero outside the grid); x neighbours come from adjacent lanes.
// The pointers are restrict-qualified so the loads of later bins can be issued early.
template <int SCM, int PPT>
__device__ __forceinline__ void update_column(const float2 (&acc)[SCM][PPT], const float2* __restrict__ Vin,
                                              float2* __restrict__ Vout, float2* __restrict__ Mm,
                                              float2* __restrict__ Mv, const UpdateArgs& u) {
    constexpr int WR = PPT + 2;
    const int n = u.n, S = u.S;
    const size_t nn = (size_t)n * n;
    const int x = u.x0 + u.lane, xc = min(x, n - 1);
    const size_t kbase = (size_t)u.kt * S * nn;
    auto load_plane = [&](int s, float2 (&w)[WR]) {
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const int y = u.y0 - 1 + r;
            w[r] = make_float2(0.f, 0.f);
            if (s >= 0 && s < S && y >= 0 && y < n) w[r] = Vin[kbase + ((size_t)s * n + y) * n + xc];
        }
    };
    if (u.ns <= 0) return;
    float2 pv[WR], cv[WR], nv[WR];
    load_plane(u.sw - 1, pv);
    load_plane(u.sw, cv);
    load_plane(u.sw + 1, nv);
#pragma unroll
    for (int q = 0; q < SCM; ++q) {
        if (q < u.ns) {
            const int s = u.sw + q;
            if (q > 0) {
#pragma unroll
                for (int r = 0; r < WR; ++r) {
                    pv[r] = cv[r];
                    cv[r] = nv[r];
                }
                load_plane(s + 1, nv);
            }
            // moments first, so their loads overlap the regulariser arithmetic
            float2 mm[PPT], vv[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const size_t idx = kbase + ((size_t)s * n + u.y0 + i) * n + xc;
                mm[i] = make_float2(0.f, 0.f);
                vv[i] = make_float2(0.f, 0.f);
                if (u.opt == VP_OPT_ADAM && u.y0 + i < n) {
                    mm[i] = Mm[idx];
                    vv[i] = Mv[idx];
                }
            }
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int y = u.y0 + i;
                if (y < n) {
                    const size_t idx = kbase + ((size_t)s * n + y) * n + xc;
                    const float2 v0 = cv[i + 1];
                    float2 left = shfl_up1(v0), right = shfl_down1(v0);
                    if (u.lane == 0) left = u.x0 > 0 ? Vin[idx - 1] : make_float2(0.f, 0.f);
                    if (u.lane == 63) right = u.x0 + 64 < n ? Vin[idx + 1] : make_float2(0.f, 0.f);
                    float2 g = make_float2(0.f, 0.f);
                    const float eps2 = u.eps2;
                    if (u.tv_w != 0.f) {
                        if (u.kt > 0) g = cadd(g, charb_w(csub(v0, Vin[idx - (size_t)S * nn]), eps2));
                        if (u.kt + 1 < u.T) g = csub(g, charb_w(csub(Vin[idx + (size_t)S * nn], v0), eps2));
                        if (s > 0) g = cadd(g, charb_w(csub(v0, pv[i + 1]), eps2));
                        if (s + 1 < S) g = csub(g, charb_w(csub(nv[i + 1], v0), eps2));
                        if (y > 0) g = cadd(g, charb_w(csub(v0, cv[i]), eps2));
                        if (y + 1 < n) g = csub(g, charb_w(csub(cv[i + 2], v0), eps2));
                        if (x > 0) g = cadd(g, charb_w(csub(v0, left), eps2));
                        if (x + 1 < n) g = csub(g, charb_w(csub(right, v0), eps2));
                        g = cscale(g, u.tv_w);
                    }
                    if (u.l1_w != 0.f) g = cfma(u.l1_w, charb_w(v0, eps2), g);
                    const float2 gr = cadd(acc[q][i], g);
                    if (x < n) {
                        float2 nvx;
                        if (u.opt == VP_OPT_ADAM) {
                            float2 m = mm[i], v = vv[i];
                            m.x = u.beta1 * m.x + (1.0f - u.beta1) * gr.x;
                            m.y = u.beta1 * m.y + (1.0f - u.beta1) * gr.y;
                            v.x = u.beta2 * v.x + (1.0f - u.beta2) * gr.x * gr.x;
                            v.y = u.beta2 * v.y + (1.0f - u.beta2) * gr.y * gr.y;
                            Mm[idx] = m;
                            Mv[idx] = v;
                            const float dx = sqrtf(v.x) * u.inv_bc2s + u.aeps;
                            const float dy = sqrtf(v.y) * u.inv_bc2s + u.aeps;
                            nvx = make_float2(v0.x - u.step_size * __fdividef(m.x, dx),
                                              v0.y - u.step_size * __fdividef(m.y, dy));
                        } else {
                            nvx = make_float2(v0.x - u.lr * gr.x, v0.y - u.lr * gr.y);
                        }
                        Vout[idx] = nvx;
                    }
                }
            }
        }
    }
}

// ------------------------------------------------------------------ adjoint gather + update
//
// G[k][s][y][x] = sum over the knot's blade parts e (plan order, blades ascending) of
//   w_e * (w00 g[y-oy][x-ox] + w01 g[y-oy][x-ox-1] + w10 g[y-oy-1][x-ox] + w11 g[y-oy-1][x-ox-1]),
// the exact transpose of k_project's taps (zero outside the grid). Work item: (knot,
// tile, chunk of 4 * sc bins); wave w owns bins s0 + w * sc ... s0 + w * sc + sc - 1.
// MODE = GATHER_STORE writes (or adds to) the gradient; GATHER_STEP adds the TV/L1
// gradient and applies the optimiser, reading volume[step & 1] and writing the other
// copy; the last finished work item of the step advances the slice's step counter.
// In the update each lane walks its column through the wave's bins with a register
// window of the previous, current and next bin (rows y0-1 .. y0+kTileRows), taking
// the x neighbours from the adjacent lanes.

template <int MODE, int SE, int P>
__global__ __launch_bounds__(kThreads) void k_gather(const KArgs a) {
    extern __shared__ float2 sm[];
    constexpr int PPT = kTileRows, SCM = kChunkMax;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int ti = blockIdx.x; ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S), T = DF(T), B = DF(B), nparts = DF(nparts), sched = DF(schedule);
        const int kt = tk->a;
        const size_t nn = (size_t)n * n;
        const int txn = (n + kTileW - 1) / kTileW;
        const int y0 = (tk->b / txn) * PPT, x0 = (tk->b % txn) * kTileW;
        const int sc = DF(gath_sc);
        const int sw = tk->c * 4 * sc + wave * sc;
        const int ns = max(0, min(sc, S - sw));
        const AS4 KnotInfo* ki = cst(DF(knots)) + kt;
        const int kox = ki->ox_max, koy = ki->oy_max;
        const int RH = PPT + koy - ki->oy_min + 1, RW = kTileW + kox - ki->ox_min + 1;
        const int RE = RH * RW;
        const AS4 KnotEntry* ent = cst(DF(knot_ent));
        const AS4 ShearEntry* shear = cst(DF(shear));
        const float2* const work = DF(work);
        const int* kp = DF(knot_ptr);
        const int e0 = cst(kp)[kt], e1 = cst(kp)[kt + 1];
        float2 acc[SCM][PPT];
#pragma unroll
        for (int q = 0; q < SCM; ++q)
#pragma unroll
            for (int i = 0; i < PPT; ++i) acc[q][i] = make_float2(0.f, 0.f);
        Stager<SE, P> sg;
        sg.init(RH, RW, y0 - koy - 1, x0 - kox - 1, n);
        float2 pre[P][SE];
        // the knot's active parts in plan order, P per phase: cur[] this phase, nxt[] the next
        auto next_active = [&](int e) {
            while (e < e1 && !active_blade(sched, stepp, st, B, ent[e].blade)) ++e;
            return e;
        };
        int cur[P];
        {
            int e = e0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                e = next_active(e);
                cur[p] = e;
                if (e < e1) ++e;
            }
            const float2* planes[P];
#pragma unroll
            for (int p = 0; p < P; ++p) planes[p] = cur[p] < e1 ? work + (size_t)ent[cur[p]].blade * nparts * nn : nullptr;
            if (cur[0] < e1) sg.fetch(planes, pre);
        }
        for (int it = 0; cur[0] < e1; ++it) {
            float2* buf = sm + (it & 1) * P * RE;
            sg.store(buf, pre);
            __syncthreads();
            int nxt[P];
            {
                int e = cur[P - 1] < e1 ? cur[P - 1] + 1 : e1;
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    e = next_active(e);
                    nxt[p] = e;
                    if (e < e1) ++e;
                }
                const float2* planes[P];
#pragma unroll
                for (int p = 0; p < P; ++p)
                    planes[p] = nxt[p] < e1 ? work + (size_t)ent[nxt[p]].blade * nparts * nn : nullptr;
                if (nxt[0] < e1) sg.fetch(planes, pre);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (cur[p] < e1) {
                    const int b = ent[cur[p]].blade;
                    const float wb = ent[cur[p]].weight;
                    const AS4 ShearEntry* shb = shear + (size_t)b * S + sw;
#pragma unroll
                    for (int q = 0; q < SCM; ++q) {
                        if (q < ns) {
                            const float w00 = shb[q].w00, w01 = shb[q].w01, w10 = shb[q].w10, w11 = shb[q].w11;
                            // row of g[y - oy][.] for pixel row 0, column of g[.][x - ox]
                            const float2* L = buf + p * RE + (koy - shb[q].oy + 1) * RW + (kox - shb[q].ox + 1) + lane;
                            float2 u0 = L[-RW], u1 = L[-RW - 1];
#pragma unroll
                            for (int i = 0; i < PPT; ++i) {
                                const float2 v0 = L[i * RW], v1 = L[i * RW - 1];
                                float2 t = make_float2(0.f, 0.f);
                                t = cfma(w00, v0, t);
                                t = cfma(w01, v1, t);
                                t = cfma(w10, u0, t);
                                t = cfma(w11, u1, t);
                                acc[q][i] = cfma(wb, t, acc[q][i]);
                                u0 = v0;
                                u1 = v1;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < P; ++p) cur[p] = nxt[p];
        }
        __syncthreads();
        const int x = x0 + lane;
        if (MODE == GATHER_STORE) {
            float2* const grad = DF(grad);
            if (x < n) {
#pragma unroll
                for (int q = 0; q < SCM; ++q) {
                    if (q < ns) {
#pragma unroll
                        for (int i = 0; i < PPT; ++i) {
                            const int y = y0 + i;
                            if (y < n) {
                                const size_t idx = (((size_t)kt * S + sw + q) * n + y) * n + x;
                                float2 g = acc[q][i];
                                if (a.accumulate) g = cadd(grad[idx], g);
                                grad[idx] = g;
                            }
                        }
                    }
                }
            }
        } else {
            const float2* const Vin = stepp ? DF(vol[st & 1]) : DF(vol[0]);
            float2* const Vout = DF(vol[(st + 1) & 1]);
            float2* const Mm = DF(m);
            float2* const Mv = DF(v);
            const int opt = DF(optimizer);
            const float lr = DF(lr), beta1 = DF(beta1), beta2 = DF(beta2), aeps = DF(adam_eps);
            const float tv_w = DF(tv_w), l1_w = DF(l1_w), teps = DF(tv_eps);
            const float eps2 = teps * teps;
            const int t = st + 1;
            // bias corrections in FP64, once per item
            const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
            const float inv_bc2s = (float)(1.0 / sqrt(1.0 - pow((double)beta2, (double)t)));
            const float step_size = lr / bc1;
            UpdateArgs u;
            u.n = n; u.S = S; u.T = T; u.kt = kt; u.y0 = y0; u.x0 = x0; u.lane = lane; u.sw = sw; u.ns = ns;
            u.opt = opt; u.lr = lr; u.beta1 = beta1; u.beta2 = beta2; u.aeps = aeps;
            u.tv_w = tv_w; u.l1_w = l1_w; u.eps2 = eps2; u.inv_bc2s = inv_bc2s; u.step_size = step_size;
            update_column<SCM, PPT>(acc, Vin, Vout, Mm, Mv, u);
            unsigned* const sync = DF(sync);
            if (sync) {
                // every work item of the slice read *step before finishing; the last one
                // to finish advances it for the next step
                const int ntask = DF(n_gath_tasks);
                __syncthreads();
                if (threadIdx.x == 0) {
                    __threadfence();
                    const unsigned prev = atomicAdd(sync, 1u);
                    if (prev + 1 == (unsigned)ntask) {
                        atomicExch(sync, 0u);
                        atomicExch(stepp, st + 1);
                    }
                }
            }
        }
    }
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
                const float q = z.x * z.x + z.y * z.y;
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

hipError_t launch_project(const KArgs& a, int gw, int re, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 g(grid_for(a.ntasks)), b(kThreads);
    const int depth = stage_depth(re);
    const size_t lds = stage_lds_bytes(re);
#define P(GW)                                                                      \
    do {                                                                           \
        if (depth == 5) hipLaunchKernelGGL((k_project<GW, 5, 3>), g, b, lds, s, a); \
        else if (depth == 8) hipLaunchKernelGGL((k_project<GW, 8, 2>), g, b, lds, s, a); \
        else hipLaunchKernelGGL((k_project<GW, 16, 1>), g, b, lds, s, a);           \
    } while (0)
    switch (gw) {
        case 1: P(1); break;
        case 2: P(2); break;
        case 4: P(4); break;
        default: P(8); break;
    }
#undef P
    return hipGetLastError();
}
hipError_t launch_rows(const KArgs& a, int dir, size_t lds, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (dir < 0)
        hipLaunchKernelGGL(k_rows<-1>, dim3(grid_for(a.ntasks)), dim3(kThreads), lds, s, a);
    else
        hipLaunchKernelGGL(k_rows<1>, dim3(grid_for(a.ntasks)), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}
hipError_t launch_cols(const KArgs& a, size_t lds, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cols, dim3(grid_for(a.ntasks)), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}
hipError_t launch_gather(const KArgs& a, int mode, int re, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 g(grid_for(a.ntasks)), b(kThreads);
    const int depth = stage_depth(re);
    const size_t lds = stage_lds_bytes(re);
#define G(MODE)                                                                      \
    do {                                                                             \
        if (depth == 5) hipLaunchKernelGGL((k_gather<MODE, 5, 3>), g, b, lds, s, a);  \
        else if (depth == 8) hipLaunchKernelGGL((k_gather<MODE, 8, 2>), g, b, lds, s, a); \
        else hipLaunchKernelGGL((k_gather<MODE, 16, 1>), g, b, lds, s, a);           \
    } while (0)
    if (mode == GATHER_STEP) G(GATHER_STEP);
    else G(GATHER_STORE);
#undef G
    return hipGetLastError();
}
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
