// The optimiser update of a lane's column (Section 4.3) that the gather kernels fuse
// into their steps and the separate update pass runs: TV (Charbonnier) and L1 gradients
// added to the data gradient, then Adam or gradient descent. Device code shared by
// k_gather.hip and k_gather_res.hip.
#pragma once

#include "kcommon.h"
#include "runtime.h"

namespace vp {

// ------------------------------------------------------------------ optimiser update of a column

struct UpdateArgs {
    int n, S, T, kt, y0, x0, lane, sw, ns, opt;
    float lr, beta1, beta2, c1, c2, aeps, tv_w, l1_w, eps2, inv_bc2s, step_size;
};


// Raw buffer load and store of one complex value at byte offsets voff (per lane) and
// soff (uniform); loads beyond the buffer read zero, stores there are dropped.
// CP is the cache-policy operand (epi_cache): 0, or non-temporal for streamed data.
template <int CP = 0>
__device__ __forceinline__ float2 buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CP));
}
template <int CP = 0>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, float2 v, int voff, int soff) {
    using v2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, v), r, voff, soff, CP);
}

// One voxel's regulariser gradient plus its data gradient `acc`, then the optimiser
// update (Section 4.3): v0 the voxel at column x, row y, with x neighbours left/right,
// time neighbours tp/tn, the Charbonnier weights of its differences with the previous
// and next bin (wsp, wsn) and row (wyp, wyn); mm, vv its Adam moments. Writes the new
// moments and value at byte offsets (vo, so) of rM, rW and rO (lanes past the grid pass
// an out-of-range vo, so their stores are dropped). The TV terms are added in a fixed
// order (t, s, y, x), so every kernel calling this gives the same bits.
template <int CP>
__device__ __forceinline__ void voxel_update(const UpdateArgs& u, bool tv, bool adam, bool l1, int x, int y,
                                             float2 v0, float2 left, float2 right, float2 tp, float2 tn, float2 wsp,
                                             float2 wsn, float2 wyp, float2 wyn, float2 acc, float2 mm, float2 vv,
                                             __amdgpu_buffer_rsrc_t rM, __amdgpu_buffer_rsrc_t rW,
                                             __amdgpu_buffer_rsrc_t rO, int vo, int so) {
    const int n = u.n;
    const float eps2 = u.eps2;
    float2 g = make_float2(-0.f, -0.f);
    if (tv) {
        if (u.kt > 0) g = cadd(g, charb_w(csub(v0, tp), eps2));
        if (u.kt + 1 < u.T) g = csub(g, charb_w(csub(tn, v0), eps2));
        g = cadd(g, wsp);
        g = csub(g, wsn);
        if (y > 0) g = cadd(g, wyp);
        if (y + 1 < n) g = csub(g, wyn);
        if (x > 0) g = cadd(g, charb_w(csub(v0, left), eps2));
        if (x + 1 < n) g = csub(g, charb_w(csub(right, v0), eps2));
        g = cscale(g, u.tv_w);
    }
    if (l1) g = cfma(u.l1_w, charb_w(v0, eps2), g);
    const float2 gr = cadd(acc, g);
    float2 nvx;
    if (adam) {
        float2 m = mm, v = vv;
        const float c1 = u.c1, c2 = u.c2;
        m.x = __builtin_fmaf(u.beta1, m.x, c1 * gr.x);
        m.y = __builtin_fmaf(u.beta1, m.y, c1 * gr.y);
        v.x = __builtin_fmaf(u.beta2, v.x, (c2 * gr.x) * gr.x);
        v.y = __builtin_fmaf(u.beta2, v.y, (c2 * gr.y) * gr.y);
        buf_st<CP>(rM, m, vo, so);
        buf_st<CP>(rW, v, vo, so);
        // hardware square root and reciprocal (about 1 ulp each)
        const float dx = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.x), u.inv_bc2s, u.aeps);
        const float dy = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.y), u.inv_bc2s, u.aeps);
        nvx = make_float2(__builtin_fmaf(-u.step_size, m.x * __builtin_amdgcn_rcpf(dx), v0.x),
                          __builtin_fmaf(-u.step_size, m.y * __builtin_amdgcn_rcpf(dy), v0.y));
    } else {
        nvx = make_float2(__builtin_fmaf(-u.lr, gr.x, v0.x), __builtin_fmaf(-u.lr, gr.y, v0.y));
    }
    buf_st<CP>(rO, nvx, vo, so);
}

// The memory side of the update of one lane's column (column x0 + lane, rows y0 ..
// y0 + PPT - 1 of knot kt): buffers over this knot's volume in each array (and the
// neighbouring knots' volumes), so that a bin's offset is scalar (soffset) and a row's
// lane offset a fixed 32-bit voffset, and no load or store needs 64-bit address
// arithmetic; rows outside the grid read zero through an out-of-range voffset.
template <int PPT, int EPI>
struct ColumnStream {
    static constexpr int WR = PPT + 2;  // window rows y0 - 1 .. y0 + PPT
    // the moments are read once and the moments and values written once per step, and an
    // item's loads of the previous knot's planes are the last of the three reads of those
    // planes (by that knot's own item and the items of the knots on either side) in every
    // work-list order: these accesses are streamed (non-temporal) when the step's state
    // does not fit the caches (EPI_STREAM), so they do not push out the planes that other
    // items read again
    static constexpr int CP = epi_cache(EPI);
    int nn, x;
    bool tv, adam, l1;
    __amdgpu_buffer_rsrc_t rV, rP, rN, rO, rM, rW;
    int rb[WR];  // byte offsets of the window rows (out of range outside the grid)
    int rs[PPT];  // store offsets of the tile's rows (out of range past the grid's last column)
    int hb;      // x halo offset of this lane (see init)

    __device__ __forceinline__ void init(const UpdateArgs& u, const float2* __restrict__ Vin,
                                         float2* __restrict__ Vout, float2* __restrict__ Mm,
                                         float2* __restrict__ Mv) {
        const int n = u.n;
        nn = n * n;
        const int kvol = u.S * nn;  // elements of one knot's volume (at most 2^26)
        const size_t kbase = (size_t)u.kt * kvol;
        x = u.x0 + u.lane;
        const int xc = min(x, n - 1);
        tv = epi_fast(EPI) || u.tv_w != 0.f;
        adam = epi_fast(EPI) || u.opt == VP_OPT_ADAM;
        l1 = !epi_fast(EPI) && u.l1_w != 0.f;
        rV = plane_rsrc(Vin + kbase, kvol);
        rP = plane_rsrc(u.kt > 0 ? Vin + kbase - kvol : Vin, u.kt > 0 ? kvol : 0);
        rN = plane_rsrc(u.kt + 1 < u.T ? Vin + kbase + kvol : Vin, u.kt + 1 < u.T ? kvol : 0);
        rO = plane_rsrc(Vout + kbase, kvol);
        rM = plane_rsrc(adam ? Mm + kbase : Vin, adam ? kvol : 0);
        rW = plane_rsrc(adam ? Mv + kbase : Vin, adam ? kvol : 0);
#pragma unroll
        for (int r = 0; r < WR; ++r) {
            const int y = u.y0 - 1 + r;
            rb[r] = (y >= 0 && y < n) ? (y * n + xc) * (int)sizeof(float2) : kBufferOut;
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) rs[i] = x < n ? rb[i + 1] : kBufferOut;
        // x halos of the tile's rows: lane i < PPT reads column x0 - 1 of row y0 + i and
        // lane 32 + i column x0 + 64 (out of range, hence zero, past the grid's border or
        // its last row); lanes 0 and 63 take them by readlane, so one load per bin serves
        // every row
        hb = kBufferOut;
        if (u.lane < PPT) {
            const int y = u.y0 + u.lane;
            if (y < n && u.x0 > 0) hb = (y * n + u.x0 - 1) * (int)sizeof(float2);
        } else if (u.lane >= 32 && u.lane < 32 + PPT) {
            const int y = u.y0 + u.lane - 32;
            if (y < n && u.x0 + 64 < n) hb = (y * n + u.x0 + 64) * (int)sizeof(float2);
        }
    }
    // Window rows of bin s (zero outside 0 .. S - 1).
    __device__ __forceinline__ void load_plane(const UpdateArgs& u, int s, float2 (&w)[WR]) const {
        if (s >= 0 && s < u.S) {
#pragma unroll
            for (int k = 0; k < WR; ++k) w[k] = buf_ld(rV, rb[k], s * nn * (int)sizeof(float2));
        } else {
#pragma unroll
            for (int k = 0; k < WR; ++k) w[k] = make_float2(0.f, 0.f);
        }
    }
    // The other loads of bin s's update: the x halos, the Adam moments (unless
    // `moments` is false: the caller has them) and the time neighbours (zero where unused).
    __device__ __forceinline__ void load_bin(const UpdateArgs& u, int s, bool moments, float2& hv, float2 (&mm)[PPT],
                                             float2 (&vv)[PPT], float2 (&tp)[PPT], float2 (&tn)[PPT]) const {
        const int so = s * nn * (int)sizeof(float2);
        hv = buf_ld(rV, hb, so);
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            tp[i] = tn[i] = make_float2(0.f, 0.f);
            if (moments) mm[i] = vv[i] = make_float2(0.f, 0.f);
            if (adam && moments) {
                mm[i] = buf_ld<CP>(rM, rb[i + 1], so);
                vv[i] = buf_ld<CP>(rW, rb[i + 1], so);
            }
            if (tv && u.kt > 0) tp[i] = buf_ld<CP>(rP, rb[i + 1], so);
            if (tv && u.kt + 1 < u.T) tn[i] = buf_ld(rN, rb[i + 1], so);
        }
    }
    // Weights of the differences between bin s (cv) and bin s + 1 (nv); zero unless both
    // bins exist.
    __device__ __forceinline__ void next_s_weights(const UpdateArgs& u, int s, const float2 (&cv)[WR],
                                                   const float2 (&nv)[WR], float2 (&wsn)[PPT]) const {
        const bool both = tv && s >= 0 && s + 1 < u.S;
#pragma unroll
        for (int i = 0; i < PPT; ++i)
            wsn[i] = both ? charb_w(csub(nv[i + 1], cv[i + 1]), u.eps2) : make_float2(0.f, 0.f);
    }
    // The update of bin s from its window cv, the s weights before (wsp) and after (wsn)
    // it, its data gradient and the loads of load_bin.
    __device__ __forceinline__ void update_bin(const UpdateArgs& u, int s, const float2 (&cv)[WR],
                                               const float2 (&wsp)[PPT], const float2 (&wsn)[PPT],
                                               const float2 (&acc)[PPT], float2 hv, const float2 (&mm)[PPT],
                                               const float2 (&vv)[PPT], const float2 (&tp)[PPT],
                                               const float2 (&tn)[PPT]) const {
        const int so = s * nn * (int)sizeof(float2);
        float2 wy[PPT + 1];
#pragma unroll
        for (int r = 0; r <= PPT; ++r) wy[r] = tv ? charb_w(csub(cv[r + 1], cv[r]), u.eps2) : make_float2(0.f, 0.f);
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int y = u.y0 + i;
            if (y < u.n) {
                const float2 v0 = cv[i + 1];
                float2 left = shfl_up1(v0), right = shfl_down1(v0);
                const float2 hl = lane_f2(hv, i), hr = lane_f2(hv, 32 + i);
                if (u.lane == 0) left = hl;
                if (u.lane == 63) right = hr;
                voxel_update<CP>(u, tv, adam, l1, x, y, v0, left, right, tp[i], tn[i], wsp[i], wsn[i], wy[i], wy[i + 1],
                             acc[i], mm[i], vv[i], rM, rW, rO, rs[i], so);
            }
        }
    }
};

// Adds the TV/L1 gradient to the data gradient acc of one lane's voxels (bins sw ..
// sw + ns - 1, rows y0 .. y0 + PPT - 1, column x0 + lane of knot kt) and applies Adam
// or GD, reading Vin and writing Vout (distinct buffers, as are the moments). The lane
// walks its bins with a register window of the previous, current and next bin (rows
// y0 - 1 .. y0 + PPT, zero outside the grid); x neighbours come from adjacent lanes.
// Each Charbonnier weight of a forward difference along s or y is computed once and
// used by both voxels of the pair (the s weight is carried to the next bin), with the
// same operands as a per-voxel evaluation, so the result is the same either way. The s
// weights of the first and last bins' outer differences are zero, so they are added
// unconditionally; the sums start from -0, which adds exactly.
template <int SCM, int PPT, int EPI, bool PRE>
__device__ __forceinline__ void update_column(const float2 (&acc)[SCM][PPT], const float2 (&pm)[SCM][PPT],
                                              const float2 (&pv)[SCM][PPT], const float2* __restrict__ Vin,
                                              float2* __restrict__ Vout, float2* __restrict__ Mm,
                                              float2* __restrict__ Mv, const UpdateArgs& u) {
    constexpr int WR = PPT + 2;
    ColumnStream<PPT, EPI> cs;
    cs.init(u, Vin, Vout, Mm, Mv);
    if (u.ns <= 0) return;
    // win[k]: rows of bin sw - 1 + k; the loop over bins is unrolled, so bin q reads
    // win[q], win[q + 1], win[q + 2] in place (no register copies between bins)
    float2 win[SCM + 2][WR];
    cs.load_plane(u, u.sw - 1, win[0]);
    cs.load_plane(u, u.sw, win[1]);
    cs.load_plane(u, u.sw + 1, win[2]);
    float2 ws[SCM + 1][PPT];  // ws[k]: weights of the differences between bins sw - 1 + k and sw + k
    cs.next_s_weights(u, u.sw - 1, win[0], win[1], ws[0]);
#pragma unroll
    for (int q = 0; q < SCM; ++q) {
        if (q < u.ns) {
            const int s = u.sw + q;
            if (q > 0) cs.load_plane(u, s + 1, win[q + 2]);
            // moments, time neighbours and x halos first, so their loads overlap the arithmetic
            float2 hv, mm[PPT], vv[PPT], tp[PPT], tn[PPT];
            if (PRE) {
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    mm[i] = pm[q][i];
                    vv[i] = pv[q][i];
                }
            }
            cs.load_bin(u, s, !PRE, hv, mm, vv, tp, tn);
            cs.next_s_weights(u, s, win[q + 1], win[q + 2], ws[q + 1]);
            cs.update_bin(u, s, win[q + 1], ws[q], ws[q + 1], acc[q], hv, mm, vv, tp, tn);
        }
    }
}

// Adam moments of a lane's voxels (the values update_column would load for them),
// loaded ahead so that their latency overlaps the gather; zero where update_column
// does not use them.
template <int SCM, int PPT, int EPI>
__device__ __forceinline__ void load_moments(const KArgs& a, int slice, int kt, int y0, int x0, int lane, int sw,
                                             int ns, float2 (&pm)[SCM][PPT], float2 (&pv)[SCM][PPT]) {
    const int n = DF(n), S = DF(S);
#pragma unroll
    for (int q = 0; q < SCM; ++q)
#pragma unroll
        for (int i = 0; i < PPT; ++i) pm[q][i] = pv[q][i] = make_float2(0.f, 0.f);
    // gradient descent keeps no moments (the arrays may be absent)
    if (!(epi_fast(EPI) || DF(optimizer) == VP_OPT_ADAM)) return;
    const int nn = n * n, kvol = S * nn;
    const size_t kbase = (size_t)kt * kvol;
    const __amdgpu_buffer_rsrc_t rM = plane_rsrc(DF(m) + kbase, kvol);
    const __amdgpu_buffer_rsrc_t rW = plane_rsrc(DF(v) + kbase, kvol);
    const int xc = min(x0 + lane, n - 1);
#pragma unroll
    for (int q = 0; q < SCM; ++q)
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int y = y0 + i;
            if (q < ns && y < n) {
                const int vo = (y * n + xc) * (int)sizeof(float2), so = (sw + q) * nn * (int)sizeof(float2);
                pm[q][i] = buf_ld<epi_cache(EPI)>(rM, vo, so);
                pv[q][i] = buf_ld<epi_cache(EPI)>(rW, vo, so);
            }
        }
}

// The update's arguments for a lane of a work item with the slice's hyperparameters at
// step st (Adam's bias corrections once per item).
__device__ __forceinline__ UpdateArgs update_args(const KArgs& a, int slice, int st, int kt, int y0, int x0, int lane,
                                                  int sw, int ns) {
    const float lr = DF(lr), teps = DF(tv_eps);
    UpdateArgs u;
    u.n = DF(n); u.S = DF(S); u.T = DF(T); u.kt = kt; u.y0 = y0; u.x0 = x0; u.lane = lane; u.sw = sw; u.ns = ns;
    u.opt = DF(optimizer); u.lr = lr; u.beta1 = DF(beta1); u.beta2 = DF(beta2); u.aeps = DF(adam_eps);
    u.c1 = 1.0f - u.beta1;
    u.c2 = 1.0f - u.beta2;
    u.tv_w = DF(tv_w); u.l1_w = DF(l1_w); u.eps2 = charb_eps2(teps);
    u.inv_bc2s = 1.f;
    u.step_size = lr;
    if (u.opt == VP_OPT_ADAM) {
        // bias corrections 1 - beta^t = -expm1(t ln beta), t = step + 1, once per item
        const float tf = (float)(st + 1);
        const float bc1 = -expm1f(tf * DF(ln_beta1)), bc2 = -expm1f(tf * DF(ln_beta2));
        u.step_size = lr / bc1;
        u.inv_bc2s = 1.f / sqrtf(bc2);
    }
    return u;
}

// Regulariser gradient and optimiser update of a lane's voxels (update_column) with the
// slice's hyperparameters (block 0 of the step's last kernel advances the step counter).
// PRE: the moments come from load_moments (pm, pv) instead of being loaded here.
template <int SCM, int PPT, int EPI, bool PRE>
__device__ __forceinline__ void update_and_finish(const KArgs& a, int slice, int* stepp, int st,
                                                  const float2 (&acc)[SCM][PPT], const float2 (&pm)[SCM][PPT],
                                                  const float2 (&pv)[SCM][PPT], int kt, int y0, int x0,
                                                  int lane, int sw, int ns) {
    const float2* const Vin = stepp ? DF(vol[st & 1]) : DF(vol[0]);
    float2* const Vout = DF(vol[(st + 1) & 1]);
    const UpdateArgs u = update_args(a, slice, st, kt, y0, x0, lane, sw, ns);
    update_column<SCM, PPT, EPI, PRE>(acc, pm, pv, Vin, Vout, DF(m), DF(v), u);
}

}  // namespace vp
