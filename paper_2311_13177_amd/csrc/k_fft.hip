// DFT passes of the lifted-PROPELLER step (Section 4.2 "Blur"): the forward row DFT
// (after blending a dynamic blade's knot projections), the column pass (forward column
// DFT, unitary scaling, blade mask, residual, loss partials, inverse column DFT) and the
// inverse row DFT, each in LDS.

#include "kcommon.h"

namespace vp {

// ------------------------------------------------------------------ DFT in LDS
//
// Mixed-radix Stockham autosort (radices 2, 3, 4, 5, and 8 in the compile-time variants), in place: in every stage each
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
        const float2 h = make_float2(__builtin_fmaf(-0.5f, t.x, x[0].x), __builtin_fmaf(-0.5f, t.y, x[0].y));
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
        const float2 p1 = make_float2(__builtin_fmaf(c2, a2.x, __builtin_fmaf(c1, a1.x, x0.x)),
                                      __builtin_fmaf(c2, a2.y, __builtin_fmaf(c1, a1.y, x0.y)));
        const float2 p2 = make_float2(__builtin_fmaf(c1, a2.x, __builtin_fmaf(c2, a1.x, x0.x)),
                                      __builtin_fmaf(c1, a2.y, __builtin_fmaf(c2, a1.y, x0.y)));
        const float2 q1 = mul_i<DIR>(make_float2(__builtin_fmaf(s2, b2.x, s1 * b1.x), __builtin_fmaf(s2, b2.y, s1 * b1.y)));
        const float2 q2 = mul_i<DIR>(make_float2(__builtin_fmaf(-s1, b2.x, s2 * b1.x), __builtin_fmaf(-s1, b2.y, s2 * b1.y)));
        x[0] = cadd(x0, cadd(a1, a2));
        x[1] = cadd(p1, q1);
        x[2] = cadd(p2, q2);
        x[3] = csub(p2, q2);
        x[4] = csub(p1, q1);
    } else if constexpr (R == 8) {
        // two 4-point DFTs (even and odd inputs), the odd ones times w^k with w the
        // eighth root of unity of the transform's sign, then the 2-point combination:
        // X[k] = E[k] + w^k O[k], X[k + 4] = E[k] - w^k O[k]
        float2 e[4] = {x[0], x[2], x[4], x[6]};
        float2 o[4] = {x[1], x[3], x[5], x[7]};
        butterfly<DIR, 4>(e);
        butterfly<DIR, 4>(o);
        const float c = 0.70710678118654752440f;  // 1 / sqrt(2)
        const float d = (float)DIR;
        const float2 o1 = make_float2(c * (o[1].x - d * o[1].y), c * (o[1].y + d * o[1].x));
        const float2 o2 = mul_i<DIR>(o[2]);
        const float2 o3 = make_float2(c * (-o[3].x - d * o[3].y), c * (-o[3].y + d * o[3].x));
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], o1);
        x[5] = csub(e[1], o1);
        x[2] = cadd(e[2], o2);
        x[6] = csub(e[2], o2);
        x[3] = cadd(e[3], o3);
        x[7] = csub(e[3], o3);
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
// arithmetic are constants. The factorisation is the plan's (4s, then 2s, 3s, 5s), so
// results equal the runtime variant's bit for bit, except for 512 points (only the
// oversampled grids of blade-aligned sampling), which take radix-8 stages (8 8 8: three
// barrier-separated stages instead of five; measured faster there, and not at 256). A
// given length always takes the same variant, whatever the kernel or batch.
__host__ __device__ constexpr int ct_radix(int n, int i) {
    int st = 0;
    if (n == 512) {
        for (; st < 3; ++st)
            if (st == i) return 8;
        return 0;
    }
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
// NC != 0: the launch holds slices of length NC only, and its compile-time plan is the
// whole transform (a kernel with just that variant needs far fewer registers).
template <int DIR, int NC = 0>
__device__ void fft_rows_any(float2* buf, const float2* tw, int n, int nstage, int code) {
    if constexpr (NC != 0) {
        ct_fft<DIR, false, NC, fft_rows_per_item(NC)>(buf, tw);
        return;
    }
    switch (n) {
        case 64: ct_fft<DIR, false, 64, fft_rows_per_item(64)>(buf, tw); break;
        case 128: ct_fft<DIR, false, 128, fft_rows_per_item(128)>(buf, tw); break;
        case 192: ct_fft<DIR, false, 192, fft_rows_per_item(192)>(buf, tw); break;
        case 256: ct_fft<DIR, false, 256, fft_rows_per_item(256)>(buf, tw); break;
        case 320: ct_fft<DIR, false, 320, fft_rows_per_item(320)>(buf, tw); break;
        case 384: ct_fft<DIR, false, 384, fft_rows_per_item(384)>(buf, tw); break;
        case 512: ct_fft<DIR, false, 512, fft_rows_per_item(512)>(buf, tw); break;
        default: lds_fft<DIR, false, 8>(buf, tw, n, fft_rows_per_item(n), n, 1, nstage, code); break;
    }
}
template <int DIR, int NC = 0>
__device__ void fft_cols_any(float2* buf, const float2* tw, int n, int nstage, int code) {
    if constexpr (NC != 0) {
        ct_fft<DIR, true, NC, fft_cols_per_item(NC)>(buf, tw);
        return;
    }
    switch (n) {
        case 64: ct_fft<DIR, true, 64, fft_cols_per_item(64)>(buf, tw); break;
        case 128: ct_fft<DIR, true, 128, fft_cols_per_item(128)>(buf, tw); break;
        case 192: ct_fft<DIR, true, 192, fft_cols_per_item(192)>(buf, tw); break;
        case 256: ct_fft<DIR, true, 256, fft_cols_per_item(256)>(buf, tw); break;
        case 320: ct_fft<DIR, true, 320, fft_cols_per_item(320)>(buf, tw); break;
        case 384: ct_fft<DIR, true, 384, fft_cols_per_item(384)>(buf, tw); break;
        case 512: ct_fft<DIR, true, 512, fft_cols_per_item(512)>(buf, tw); break;
        default: {
            const int cb = fft_cols_per_item(n);
            lds_fft<DIR, true, 16>(buf, tw, n, cb, 1, cb, nstage, code);
            break;
        }
    }
}

// ------------------------------------------------------------------ row passes
//
// DIR = -1: blend the blade's knot projections, (1 - a) P_k + a P_{k+1}, and take the
// forward DFT of each row. DIR = +1: inverse DFT of each row (the column pass has
// already applied both unitary scalings).

template <int DIR, int NC>
__global__ __launch_bounds__(kThreads) void k_rows(const KArgs a) {
    extern __shared__ float2 sm[];
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int b = tk->a;
        if (!active_blade(DF(schedule), DF(sched_seed), stepp, st, DF(B), b)) continue;
        const int n = DF(n), nparts = DF(nparts), nstage = DF(nstage), code = DF(radix_code);
        const size_t nn = (size_t)n * n;
        const int fb = fft_rows_per_item(n);
        const int r0 = tk->b, rows = min(fb, n - r0);
        float2* A = sm;
        float2* tw = sm + fb * n;
        float2* img = (a.mode == COL_INVERSE || a.mode == COL_RAW_FWD) ? a.out0 + (size_t)b * nn
                                                                         : DF(work) + (size_t)b * nparts * nn;
        const float2* twg = DF(tw);
        const size_t base = (size_t)r0 * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
        // blade-aligned passes: grid row g holds image row (or column) g + m/2 (g < m - m/2)
        // or g - n + m/2 (g >= n - m/2) of a centred m x m image, else zero
        const int m = a.live_n, mh = m / 2;
        const bool edge = m != 0 && (a.mode == COL_INVERSE || a.mode == COL_RAW_FWD);
        if (DIR < 0 && edge) {
            const NuEdge& ne = a.nue;
            const size_t mm = (size_t)m * m;
            const float2* src = ne.img_in + (size_t)b * ne.parts * mm;
            const BladeDev bd = ne.blade[b];
            for (int i = threadIdx.x; i < fb * n; i += blockDim.x) {
                const int k = i / n, g = i - k * n, gy = r0 + k;
                const int y = gy < m - mh ? gy + mh : (gy >= n - mh ? gy - n + mh : -1);
                const int x = g < m - mh ? g + mh : (g >= n - mh ? g - n + mh : -1);
                float2 v = make_float2(0.f, 0.f);
                if (k < rows && y >= 0 && x >= 0) {
                    const float2* p = src + (size_t)y * m + x;
                    if (ne.parts == 2) {
                        if (bd.has0) v = cscale(p[0], bd.w0);
                        if (bd.has1) v = cfma(bd.w1, p[mm], v);
                    } else {
                        v = p[0];
                    }
                    v = cscale(v, ne.dea[x] * ne.dea[y]);
                }
                A[i] = v;
            }
        } else if (DIR < 0 && nparts == 2) {
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
        fft_rows_any<DIR, NC>(A, tw, n, nstage, code);
        if (DIR > 0 && edge) {
            const NuEdge& ne = a.nue;
            float2* dst = ne.img_out + (size_t)b * ne.parts * m * m;
            for (int i = threadIdx.x; i < rows * m; i += blockDim.x) {
                const int k = i / m, x = i - k * m, gy = r0 + k;
                const int y = gy < m - mh ? gy + mh : (gy >= n - mh ? gy - n + mh : -1);
                const int g = x < mh ? x - mh + n : x - mh;
                if (y >= 0) dst[(size_t)y * m + x] = cscale(A[k * n + g], ne.dea[x] * ne.dea[y]);
            }
        } else {
            for (int i = threadIdx.x; i < rows * n; i += blockDim.x) img[base + i] = A[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ column pass
//
// COL_STEP:    forward column DFT, K = X / n, R = M (K - y), loss partial w |R|^2,
//              Z = w R / n, inverse column DFT -> work (one pass per column strip; w is
//              the slice's data-term weight).
// COL_FORWARD: forward column DFT, out = M (K - y) (y optional), no inverse.
// COL_ADJOINT: reads caller k-space, Z = M kres / n, inverse column DFT -> work.
// COL_INVERSE: inverse column DFT of caller frames, unmasked and unscaled, -> a.out0.
// COL_RAW_FWD: forward column DFT of caller frames, unmasked and unscaled, -> a.out0.

template <int NC>
__global__ __launch_bounds__(kThreads) void k_cols(const KArgs a) {
    extern __shared__ float2 sm[];
    __shared__ float red[kThreads / 64];
    // Compile-time lengths keep each thread's measurement values and mask bytes in
    // registers (loaded with the strip, used after the forward DFT); the generic length
    // stages them in LDS beside the strip.
    constexpr bool kRegs = NC != 0;
    constexpr int kEpt = kRegs ? (NC * fft_cols_per_item(NC) + kThreads - 1) / kThreads : 1;
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int b = tk->a;
        float* const loss_part = DF(loss_part);
        const int n_col_items = DF(n_col_items);
        if (!active_blade(DF(schedule), DF(sched_seed), stepp, st, DF(B), b)) {
            if (a.mode == COL_STEP && threadIdx.x == 0) loss_part[b * n_col_items + tk->b] = 0.f;
            continue;
        }
        const int n = kRegs ? NC : DF(n);
        const int nparts = DF(nparts), nstage = DF(nstage), code = DF(radix_code);
        const size_t nn = (size_t)n * n;
        const int cb = fft_cols_per_item(n);
        const int c0 = tk->b * cb, cols = min(cb, n - c0);
        const int ne = n * cb;
        // LDS: the strip (cb columns of n) and the twiddles (plus, for the generic length,
        // the strip's measurement and mask), all loaded in one pass so that their
        // latencies overlap
        float2* A = sm;
        float2* tw = sm + cb * n;
        float2* Y = tw + n;
        uint8_t* M = reinterpret_cast<uint8_t*>(Y + cb * n);
        float2 yr[kEpt];
        uint8_t mr[kEpt];
        float2* img = DF(work) + (size_t)b * nparts * nn;
        const float2* twg = DF(tw);
        const bool raw = a.mode == COL_INVERSE || a.mode == COL_RAW_FWD;
        const bool from_in = a.mode == COL_ADJOINT || raw;
        const float2* src = from_in ? a.in0 + (size_t)b * nn : img;
        float2* dst = raw ? a.out0 + (size_t)b * nn : img;
        const uint8_t* mk = DF(mask) + (size_t)b * nn;
        const float2* yy = DF(y);
        const float2* yb = (yy && !from_in) ? yy + (size_t)b * nn : nullptr;
        // rows of a centred image of size live_n (all rows when 0)
        const int lv = raw ? a.live_n : 0, lv_lo = lv - lv / 2, lv_hi = n - lv / 2;
        for (int i = threadIdx.x; i < n; i += blockDim.x) tw[i] = twg[i];
        auto load = [&](int i, float2& w, uint8_t& m) {
            const int y = i / cb, c = i - (i / cb) * cb;
            float2 v = make_float2(0.f, 0.f);
            w = v;
            m = 0;
            if (c < cols) {
                const size_t gi = (size_t)y * n + c0 + c;
                if (raw) {
                    // a raw forward pass of a centred image reads only its rows
                    if (a.mode == COL_INVERSE || lv == 0 || y < lv_lo || y >= lv_hi) v = src[gi];
                } else {
                    v = src[gi];
                    m = mk[gi];
                    if (yb) w = yb[gi];
                }
            }
            A[i] = v;
        };
        if constexpr (kRegs) {
#pragma unroll
            for (int k = 0; k < kEpt; ++k) {
                const int i = threadIdx.x + k * kThreads;
                yr[k] = make_float2(0.f, 0.f);
                mr[k] = 0;
                if (kEpt * kThreads == NC * fft_cols_per_item(NC) || i < ne) load(i, yr[k], mr[k]);
            }
        } else {
            for (int i = threadIdx.x; i < ne; i += blockDim.x) {
                float2 w;
                uint8_t m;
                load(i, w, m);
                if (!raw) {
                    Y[i] = w;
                    M[i] = m;
                }
            }
        }
        __syncthreads();
        if (!from_in || a.mode == COL_RAW_FWD) fft_cols_any<-1, NC>(A, tw, n, nstage, code);
        const float sc = 1.0f / (float)n;
        // the step's residual and loss carry the data-term weight
        const float dw = a.mode == COL_STEP ? DF(data_w) : 1.0f;
        const float sc_res = dw * sc;
        float lsum = 0.f;
        auto mask_res = [&](int i, float2 yv, uint8_t mv) {
            const int y = i / cb, c = i - (i / cb) * cb;
            float2 v = make_float2(0.f, 0.f);
            if (c < cols) {
                const bool on = mv != 0;
                const float2 x = A[i];
                if (a.mode == COL_ADJOINT) {
                    if (on) v = cscale(x, sc);
                } else {
                    float2 r = make_float2(0.f, 0.f);
                    if (on) r = csub(cscale(x, sc), yv);
                    if (a.mode == COL_FORWARD) {
                        a.out0[(size_t)b * nn + (size_t)y * n + c0 + c] = r;
                    } else {
                        lsum = __builtin_fmaf(r.x, r.x, lsum);
                        lsum = __builtin_fmaf(r.y, r.y, lsum);
                        v = cscale(r, sc_res);
                    }
                }
            }
            A[i] = v;
        };
        if (!raw) {
            if constexpr (kRegs) {
#pragma unroll
                for (int k = 0; k < kEpt; ++k) {
                    const int i = threadIdx.x + k * kThreads;
                    if (kEpt * kThreads == NC * fft_cols_per_item(NC) || i < ne) mask_res(i, yr[k], mr[k]);
                }
            } else {
                for (int i = threadIdx.x; i < ne; i += blockDim.x) mask_res(i, Y[i], M[i]);
            }
        }
        __syncthreads();
        if (a.mode != COL_FORWARD) {
            if (a.mode != COL_RAW_FWD) fft_cols_any<1, NC>(A, tw, n, nstage, code);
            // a raw inverse pass feeding a centred crop writes only its rows
            const bool all = a.mode != COL_INVERSE || lv == 0;
            for (int i = threadIdx.x; i < ne; i += blockDim.x) {
                const int y = i / cb, c = i - (i / cb) * cb;
                if (c < cols && (all || y < lv_lo || y >= lv_hi)) dst[(size_t)y * n + c0 + c] = A[i];
            }
        }
        if (a.mode == COL_STEP) {
            // loss partial: butterfly sum within each wave, then the four wave sums in order
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
            __syncthreads();
            if (threadIdx.x == 0) loss_part[b * n_col_items + tk->b] = dw * ((red[0] + red[1]) + (red[2] + red[3]));
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int ntasks) { return ntasks < 1 ? 1 : (ntasks > (1 << 20) ? (1 << 20) : ntasks); }

// n: the common length of every slice of the launch (0 if they differ).
hipError_t launch_rows(const KArgs& a, int dir, int n, size_t lds, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 g(grid_for(a.ntasks)), b(kThreads);
#define RV(N)                                                                      \
    case N:                                                                        \
        if (dir < 0) hipLaunchKernelGGL((k_rows<-1, N>), g, b, lds, s, a);         \
        else hipLaunchKernelGGL((k_rows<1, N>), g, b, lds, s, a);                  \
        break
    switch (n) {
        RV(64); RV(128); RV(192); RV(256); RV(320); RV(384); RV(512);
        default: RV(0);
    }
#undef RV
    return hipGetLastError();
}
hipError_t launch_cols(const KArgs& a, int n, size_t lds, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 g(grid_for(a.ntasks)), b(kThreads);
    // the compile-time lengths hold the measurement and mask in registers: LDS for the
    // strip and the twiddles only
    if (n == 64 || n == 128 || n == 192 || n == 256 || n == 320 || n == 384 || n == 512)
        lds = (size_t)fft_cols_raw_lds(n);
#define CV(N)                                                  \
    case N:                                                    \
        hipLaunchKernelGGL((k_cols<N>), g, b, lds, s, a);      \
        break
    switch (n) {
        CV(64); CV(128); CV(192); CV(256); CV(320); CV(384); CV(512);
        default: CV(0);
    }
#undef CV
    return hipGetLastError();
}

}  // namespace vp
