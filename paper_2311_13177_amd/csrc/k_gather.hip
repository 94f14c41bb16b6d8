// Adjoint of the projection as a gather, fused with the regulariser gradient and the
// optimiser update (Sections 4.2 and 4.3).

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
__device__ __forceinline__ float2 buf_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, float2 v, int voff, int soff) {
    using v2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, v), r, voff, soff, 0);
}

// One voxel's regulariser gradient plus its data gradient `acc`, then the optimiser
// update (Section 4.3): v0 the voxel at column x, row y, with x neighbours left/right,
// time neighbours tp/tn, the Charbonnier weights of its differences with the previous
// and next bin (wsp, wsn) and row (wyp, wyn); mm, vv its Adam moments. Writes the new
// moments and value at byte offsets (vo, so) of rM, rW and rO (lanes past the grid pass
// an out-of-range vo, so their stores are dropped). The TV terms are added in a fixed
// order (t, s, y, x), so every kernel calling this gives the same bits.
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
        buf_st(rM, m, vo, so);
        buf_st(rW, v, vo, so);
        // hardware square root and reciprocal (about 1 ulp each)
        const float dx = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.x), u.inv_bc2s, u.aeps);
        const float dy = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.y), u.inv_bc2s, u.aeps);
        nvx = make_float2(__builtin_fmaf(-u.step_size, m.x * __builtin_amdgcn_rcpf(dx), v0.x),
                          __builtin_fmaf(-u.step_size, m.y * __builtin_amdgcn_rcpf(dy), v0.y));
    } else {
        nvx = make_float2(__builtin_fmaf(-u.lr, gr.x, v0.x), __builtin_fmaf(-u.lr, gr.y, v0.y));
    }
    buf_st(rO, nvx, vo, so);
}

// The memory side of the update of one lane's column (column x0 + lane, rows y0 ..
// y0 + PPT - 1 of knot kt): buffers over this knot's volume in each array (and the
// neighbouring knots' volumes), so that a bin's offset is scalar (soffset) and a row's
// lane offset a fixed 32-bit voffset, and no load or store needs 64-bit address
// arithmetic; rows outside the grid read zero through an out-of-range voffset.
template <int PPT, int EPI>
struct ColumnStream {
    static constexpr int WR = PPT + 2;  // window rows y0 - 1 .. y0 + PPT
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
        tv = EPI == EPI_ADAM_TV || u.tv_w != 0.f;
        adam = EPI == EPI_ADAM_TV || u.opt == VP_OPT_ADAM;
        l1 = EPI != EPI_ADAM_TV && u.l1_w != 0.f;
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
                mm[i] = buf_ld(rM, rb[i + 1], so);
                vv[i] = buf_ld(rW, rb[i + 1], so);
            }
            if (tv && u.kt > 0) tp[i] = buf_ld(rP, rb[i + 1], so);
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
                voxel_update(u, tv, adam, l1, x, y, v0, left, right, tp[i], tn[i], wsp[i], wsn[i], wy[i], wy[i + 1],
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
    if (!(EPI == EPI_ADAM_TV || DF(optimizer) == VP_OPT_ADAM)) return;
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
                pm[q][i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rM, vo, so, 0));
                pv[q][i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rW, vo, so, 0));
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

// ------------------------------------------------------------------ adjoint gather + update
//
// G[k][s][y][x] = sum over the knot's blade parts e (plan order, blades ascending) of
//   w_e * (w00 g[y-oy][x-ox] + w01 g[y-oy][x-ox-1] + w10 g[y-oy-1][x-ox] + w11 g[y-oy-1][x-ox-1]),
// the exact transpose of k_project's taps (zero outside the grid), accumulated tap by
// tap with the products w_e w.. from the plan's per-entry tap table. Work item: (knot,
// tile of 64 x PPT, chunk of NW * SCM bins), NW waves (4 or 8) sharing the staged blade
// regions; wave w owns bins s0 + w * SCM ... s0 + w * SCM + SCM - 1.
// MODE = GATHER_STORE writes (or adds to) the gradient; GATHER_STEP adds the TV/L1
// gradient and applies the optimiser, reading volume[step & 1] and writing the other
// copy.
// In the update each lane walks its column through the wave's bins with a register
// window of the previous, current and next bin (rows y0-1 .. y0+PPT), taking
// the x neighbours from the adjacent lanes.

// At least four waves per SIMD (at most 128 VGPRs): enough loads in flight for the
// streaming epilogue; more waves would force spills.
template <int MODE, int PPT, int SCM, int SE, int P, int EPI, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4))) void k_gather(const KArgs a) {
    extern __shared__ float2 sm[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // only a fused step ends a step here (a storing gather leaves it to the update pass);
    // compiled into the step variants alone, so the storing ones keep their registers
    if constexpr (MODE == GATHER_STEP) {
        if (a.advance) step_advance(a);
    }
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step_at(stepp, a.snap);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S), T = DF(T), B = DF(B), nparts = DF(nparts), sched = DF(schedule);
        const unsigned sseed = DF(sched_seed);
        const int kt = tk->a;
        const size_t nn = (size_t)n * n;
        const int txn = (n + kTileW - 1) / kTileW;
        const int y0 = (tk->b / txn) * PPT, x0 = (tk->b % txn) * kTileW;
        const int sw = tk->c * NW * SCM + wave * SCM;
        const int ns = max(0, min(SCM, S - sw));
        const AS4 KnotInfo* ki = cst(DF(knots)) + kt;
        const int kox = ki->ox_max, koy = ki->oy_max;
        const int RH = PPT + koy - ki->oy_min + 1, RW = kTileW + kox - ki->ox_min + 1;
        const int RE = RH * RW;
        const AS4 KnotEntry* ent = cst(DF(knot_ent));
        const AS4 ShearEntry* ktap = cst(DF(knot_tap));
        const float2* const work = DF(work);
        const int* kp = DF(knot_ptr);
        const int e0 = cst(kp)[kt], e1 = cst(kp)[kt + 1];
        float2 acc[SCM][PPT];
#pragma unroll
        for (int q = 0; q < SCM; ++q)
#pragma unroll
            for (int i = 0; i < PPT; ++i) acc[q][i] = make_float2(0.f, 0.f);
        Stager<SE, P, 64 * NW> sg;
        sg.init(RH, RW, y0 - koy - 1, x0 - kox - 1, n);
        float2 pre[P][SE];
        // the knot's active parts in plan order, P per phase: cur[] this phase, nxt[] the next
        auto next_active = [&](int e) {
            while (e < e1 && !active_blade(sched, sseed, stepp, st, B, ent[e].blade)) ++e;
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
            if (cur[0] < e1) sg.fetch(planes, (int)nn, pre);
        }
        // Adam moments loaded ahead where the registers allow (at most 128 with spills
        // of a few registers at most; larger tiles load them in the epilogue)
        constexpr bool kPre = MODE == GATHER_STEP && PPT == 2 && SCM <= 4;
        float2 pm[SCM][PPT], pv[SCM][PPT];
        if (kPre) load_moments<SCM, PPT, EPI>(a, slice, kt, y0, x0, lane, sw, ns, pm, pv);
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
                if (nxt[0] < e1) sg.fetch(planes, (int)nn, pre);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                if (cur[p] < e1) {
                    // taps of all of the wave's bins, already times the part's time weight,
                    // loaded before any is used (bins past S read the last bin's entry and
                    // are skipped)
                    const AS4 ShearEntry* shb = ktap + (size_t)cur[p] * S;
                    int tox[SCM], toy[SCM];
                    float tw[SCM][4];
#pragma unroll
                    for (int q = 0; q < SCM; ++q) {
                        const AS4 ShearEntry* sh = shb + min(sw + q, S - 1);
                        tox[q] = sh->ox;
                        toy[q] = sh->oy;
                        tw[q][0] = sh->w00;
                        tw[q][1] = sh->w01;
                        tw[q][2] = sh->w10;
                        tw[q][3] = sh->w11;
                    }
#pragma unroll
                    for (int q = 0; q < SCM; ++q) {
                        if (q < ns) {
                            const float w00 = tw[q][0], w01 = tw[q][1], w10 = tw[q][2], w11 = tw[q][3];
                            // row of g[y - oy][.] for pixel row 0, column of g[.][x - ox]
                            // row of g[y - oy][.] for pixel row 0, column of g[.][x - ox]
                            const float2* L = buf + p * RE + (koy - toy[q] + 1) * RW + (kox - tox[q] + 1) + lane;
                            float2 u0 = L[-RW], u1 = L[-RW - 1];
#pragma unroll
                            for (int i = 0; i < PPT; ++i) {
                                const float2 v0 = L[i * RW], v1 = L[i * RW - 1];
                                float2 t = acc[q][i];
                                t = cfma(w00, v0, t);
                                t = cfma(w01, v1, t);
                                t = cfma(w10, u0, t);
                                t = cfma(w11, u1, t);
                                acc[q][i] = t;
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
            update_and_finish<SCM, PPT, EPI, kPre>(a, slice, stepp, st, acc, pm, pv, kt, y0, x0, lane, sw, ns);
        }
    }
}

// ------------------------------------------------------------------ resident-parts gather + update
//
// The fused step of k_gather<GATHER_STEP> for knots whose blade parts all fit in LDS at
// once. The item (knot, tile of 64 x PPT, NW * SCM bins) stages every part's region of
// its tile in one phase (one barrier); then each wave walks its bins, and for each bin
// issues the loads of that bin's update (volume window, x halos, moments, time
// neighbours), gathers the bin's data gradient from LDS, and updates the bin. So each
// wave streams HBM while it does its own LDS and vector work, instead of every item
// gathering first and streaming afterwards. The sums run in the same order as in
// k_gather (parts in plan order, the four taps in order, then ColumnStream's update), so
// the two kernels give the same bits.
constexpr int kResTapGroup = 4;  // parts whose taps are loaded together
template <int MODE, int PPT, int SCM, int SE, int PG, int EPI, int NW, int WPE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE))) void k_gather_res(const KArgs a) {
    extern __shared__ float2 sm[];
    constexpr int NT = 64 * NW, WR = PPT + 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (MODE == GATHER_STEP) {
        if (a.advance) step_advance(a);
    }
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step_at(stepp, a.snap);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S), B = DF(B), nparts = DF(nparts), sched = DF(schedule);
        const unsigned sseed = DF(sched_seed);
        const int kt = tk->a;
        const int nn = n * n;
        const int txn = (n + kTileW - 1) / kTileW;
        const int y0 = (tk->b / txn) * PPT, x0 = (tk->b % txn) * kTileW;
        const int sw = tk->c * NW * SCM + wave * SCM;
        const int ns = max(0, min(SCM, S - sw));
        const AS4 KnotInfo* ki = cst(DF(knots)) + kt;
        const int kox = ki->ox_max, koy = ki->oy_max;
        const int RH = PPT + koy - ki->oy_min + 1, RW = kTileW + kox - ki->ox_min + 1;
        const int RE = RH * RW;
        const AS4 KnotEntry* ent = cst(DF(knot_ent));
        const AS4 ShearEntry* ktap = cst(DF(knot_tap));
        const float2* const work = DF(work);
        const int* kp = DF(knot_ptr);
        const int e0 = cst(kp)[kt], np = cst(kp)[kt + 1] - e0;  // np <= 32 (the layout checks)
        // the parts that take part in this step (all, unless a one-blade schedule runs)
        unsigned act = 0;
        for (int j = 0; j < np; ++j)
            if (active_blade(sched, sseed, stepp, st, B, ent[e0 + j].blade)) act |= 1u << j;
        // every active part's region of the tile, part j at sm[j * RE] (an inactive part's
        // region is zeros): PG parts' loads in flight at a time, each thread holding region
        // elements threadIdx.x + k * NT
        {
            Stager<SE, PG, NT> sg;
            sg.init(RH, RW, y0 - koy - 1, x0 - kox - 1, n);
            for (int j0 = 0; j0 < np; j0 += PG) {
                const float2* planes[PG];
#pragma unroll
                for (int p = 0; p < PG; ++p) {
                    const int j = j0 + p;
                    planes[p] = (j < np && ((act >> j) & 1u)) ? work + (size_t)ent[e0 + j].blade * nparts * nn : nullptr;
                }
                float2 pre[PG][SE];
                sg.fetch(planes, nn, pre);
#pragma unroll
                for (int p = 0; p < PG; ++p)
                    if (j0 + p < np)
#pragma unroll
                        for (int k = 0; k < SE; ++k)
                            if (sg.off[k] != -2) sm[(j0 + p) * RE + threadIdx.x + k * NT] = pre[p][k];
            }
        }
        __syncthreads();
        // The data gradient of bin s: parts in plan order, taps
        // w00 g[y-oy][x-ox] + w01 g[y-oy][x-ox-1] + w10 g[y-oy-1][x-ox] + w11 g[y-oy-1][x-ox-1].
        // Parts go kResTapGroup at a time, every load of a group issued before any is used.
        // A group's slots past the last part repeat the last part with zero weights, and an
        // inactive part's region is zeros: such terms add a zero to the sum, which leaves it
        // unchanged bit for bit (it starts at +0 and a sum of finite products is never -0),
        // so the sum equals the one over the active parts alone.
        auto gather_bin = [&](int s, float2 (&acc)[PPT]) {
#pragma unroll
            for (int i = 0; i < PPT; ++i) acc[i] = make_float2(0.f, 0.f);
            const AS4 ShearEntry* const tb = ktap + (size_t)e0 * S + s;
            for (int j0 = 0; j0 < np; j0 += kResTapGroup) {
                int tof[kResTapGroup];
                float tw[kResTapGroup][4];
#pragma unroll
                for (int p = 0; p < kResTapGroup; ++p) {
                    const bool real = j0 + p < np;
                    const int j = real ? j0 + p : np - 1;
                    const AS4 ShearEntry* sh = tb + j * S;
                    tof[p] = j * RE + (koy - sh->oy + 1) * RW + (kox - sh->ox + 1);
                    tw[p][0] = real ? sh->w00 : 0.f;
                    tw[p][1] = real ? sh->w01 : 0.f;
                    tw[p][2] = real ? sh->w10 : 0.f;
                    tw[p][3] = real ? sh->w11 : 0.f;
                }
#pragma unroll
                for (int p = 0; p < kResTapGroup; ++p) {
                    const float2* L = sm + tof[p] + lane;
                    float2 u0 = L[-RW], u1 = L[-RW - 1];
#pragma unroll
                    for (int i = 0; i < PPT; ++i) {
                        const float2 v0 = L[i * RW], v1 = L[i * RW - 1];
                        float2 t = acc[i];
                        t = cfma(tw[p][0], v0, t);
                        t = cfma(tw[p][1], v1, t);
                        t = cfma(tw[p][2], u0, t);
                        t = cfma(tw[p][3], u1, t);
                        acc[i] = t;
                        u0 = v0;
                        u1 = v1;
                    }
                }
            }
        };
        if constexpr (MODE == GATHER_STORE) {
            // write (or add to) the gradient, as k_gather<GATHER_STORE> does
            float2* const grad = DF(grad);
            const int x = x0 + lane;
#pragma unroll
            for (int q = 0; q < SCM; ++q) {
                if (q < ns) {
                    const int s = sw + q;
                    float2 acc[PPT];
                    gather_bin(s, acc);
                    if (x < n) {
#pragma unroll
                        for (int i = 0; i < PPT; ++i) {
                            const int y = y0 + i;
                            if (y < n) {
                                const size_t idx = (((size_t)kt * S + s) * n + y) * n + x;
                                float2 g = acc[i];
                                if (a.accumulate) g = cadd(grad[idx], g);
                                grad[idx] = g;
                            }
                        }
                    }
                }
            }
        } else if (ns > 0) {
            const float2* const Vin = stepp ? DF(vol[st & 1]) : DF(vol[0]);
            float2* const Vout = DF(vol[(st + 1) & 1]);
            const UpdateArgs u = update_args(a, slice, st, kt, y0, x0, lane, sw, ns);
            ColumnStream<PPT, EPI> cs;
            cs.init(u, Vin, Vout, DF(m), DF(v));
            // window of the current bin (cw) and the next (nw); s weights with the previous bin
            float2 cw[WR], nw[WR], wsp[PPT];
            {
                float2 pw[WR];
                cs.load_plane(u, sw - 1, pw);
                cs.load_plane(u, sw, cw);
                cs.load_plane(u, sw + 1, nw);
                cs.next_s_weights(u, sw - 1, pw, cw, wsp);
            }
#pragma unroll
            for (int q = 0; q < SCM; ++q) {
                if (q < ns) {
                    const int s = sw + q;
                    // this bin's update loads and the window of the bin after the next,
                    // issued before the gather
                    float2 fw[WR];
                    if (q + 1 < ns) {
                        cs.load_plane(u, s + 2, fw);
                    } else {
#pragma unroll
                        for (int k = 0; k < WR; ++k) fw[k] = make_float2(0.f, 0.f);
                    }
                    float2 hv, mm[PPT], vv[PPT], tp[PPT], tn[PPT];
                    cs.load_bin(u, s, true, hv, mm, vv, tp, tn);
                    float2 acc[PPT];
                    gather_bin(s, acc);
                    float2 wsn[PPT];
                    cs.next_s_weights(u, s, cw, nw, wsn);
                    cs.update_bin(u, s, cw, wsp, wsn, acc, hv, mm, vv, tp, tn);
#pragma unroll
                    for (int i = 0; i < PPT; ++i) wsp[i] = wsn[i];
#pragma unroll
                    for (int k = 0; k < WR; ++k) {
                        cw[k] = nw[k];
                        nw[k] = fw[k];
                    }
                }
            }
        }
        __syncthreads();  // the next item restages the LDS
    }
}

// ------------------------------------------------------------------ separate update pass
//
// The same update as the fused epilogue, for a data gradient G that the gather has
// stored ([T][S][n][n], in DF(grad)): G is read back exactly, and update_column does the
// same arithmetic, so the result equals the fused one bit for bit. Work item: (knot,
// block of 4 rows x 64 columns, chunk of SC bins); wave w takes row 4 * b + w. Its light
// register footprint keeps many waves in flight on what is a streaming pass.

template <int SC, int EPI>
__global__ __launch_bounds__(kThreads) void k_update(const KArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.advance) step_advance(a);
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step_at(stepp, a.snap);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S);
        const int kt = tk->a;
        const int txn = (n + kTileW - 1) / kTileW;
        const int y = (tk->b / txn) * 4 + wave, x0 = (tk->b % txn) * kTileW;
        const int sw = tk->c * SC;
        const int ns = y < n ? max(0, min(SC, S - sw)) : 0;
        const size_t nn = (size_t)n * n;
        const int off = min(y, n - 1) * n + min(x0 + lane, n - 1);
        const float2* const G = DF(grad) + (size_t)kt * S * nn;
        float2 acc[SC][1];
#pragma unroll
        for (int q = 0; q < SC; ++q) acc[q][0] = G[(size_t)min(sw + q, S - 1) * nn + off];
        update_and_finish<SC, 1, EPI, false>(a, slice, stepp, st, acc, acc, acc, kt, y, x0, lane, sw, ns);
    }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int ntasks) { return ntasks < 1 ? 1 : (ntasks > (1 << 20) ? (1 << 20) : ntasks); }

// The staging depth (planes per phase, elements per thread) follows the region size as
// for 256 threads; 512 threads need half the elements each (rounded up).
template <int MODE, int PPT, int SCM, int EPI>
static void gather_variant(const KArgs& a, int waves, int re, hipStream_t s) {
    const dim3 g(grid_for(a.ntasks)), b(64 * waves);
    const int depth = stage_depth(re);
    const size_t lds = stage_lds_bytes(re);
    if (waves == 8) {
        if (depth == 5) hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 3, 3, EPI, 8>), g, b, lds, s, a);
        else if (depth == 8) hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 4, 2, EPI, 8>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 8, 1, EPI, 8>), g, b, lds, s, a);
    } else {
        if (depth == 5) hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 5, 3, EPI, 4>), g, b, lds, s, a);
        else if (depth == 8) hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 8, 2, EPI, 4>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_gather<MODE, PPT, SCM, 16, 1, EPI, 4>), g, b, lds, s, a);
    }
}

template <int MODE>
static hipError_t gather_mode(const KArgs& a, int rows, int sc, int waves, int re, hipStream_t s) {
#define GV(R, C)                                                     \
    case R * 16 + C:                                                 \
        if constexpr (MODE == GATHER_STEP) {                         \
            if (a.epi == EPI_ADAM_TV)                                \
                gather_variant<MODE, R, C, EPI_ADAM_TV>(a, waves, re, s);   \
            else                                                     \
                gather_variant<MODE, R, C, EPI_GENERIC>(a, waves, re, s);   \
        } else {                                                     \
            gather_variant<MODE, R, C, EPI_GENERIC>(a, waves, re, s);       \
        }                                                            \
        break
    switch (rows * 16 + sc) {
        GV(2, 1); GV(2, 2); GV(2, 4); GV(2, 8);
        GV(4, 1); GV(4, 2); GV(4, 4);
        default: return hipErrorInvalidValue;
    }
#undef GV
    return hipGetLastError();
}

hipError_t launch_update(const KArgs& a, int sc, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    const dim3 g(grid_for(a.ntasks)), b(kThreads);
    const bool fast = a.epi == EPI_ADAM_TV;
#define UV(SC)                                                                          \
    case SC:                                                                            \
        if (fast) hipLaunchKernelGGL((k_update<SC, EPI_ADAM_TV>), g, b, 0, s, a);       \
        else hipLaunchKernelGGL((k_update<SC, EPI_GENERIC>), g, b, 0, s, a);            \
        break
    switch (sc) {
        UV(2); UV(4); UV(8);
        default: return hipErrorInvalidValue;
    }
#undef UV
    return hipGetLastError();
}

// Resident-parts variants: PG parts staged per phase, SE elements per thread covering
// the largest region re (at most kResRegion elements): the steps take half the elements
// per thread (fewer staging registers) where the regions are at most half as large.
template <int MODE, int PPT, int SCM, int EPI>
static void gather_res_variant(const KArgs& a, int waves, int re, size_t lds, hipStream_t s) {
    const dim3 g(grid_for(a.ntasks)), b(64 * waves);
    // two-row tiles fit five waves per SIMD (at most 102 VGPRs), four-row tiles four
    constexpr int WPE = PPT == 2 ? 5 : 4;
    const bool half = MODE == GATHER_STEP && re <= kResRegion / 2;
    if (waves == 8) {
        if (half) hipLaunchKernelGGL((k_gather_res<MODE, PPT, SCM, kResRegion / 1024, 4, EPI, 8, WPE>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_gather_res<MODE, PPT, SCM, kResRegion / 512, 4, EPI, 8, WPE>), g, b, lds, s, a);
    } else {
        if (half) hipLaunchKernelGGL((k_gather_res<MODE, PPT, SCM, kResRegion / 512, 4, EPI, 4, WPE>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_gather_res<MODE, PPT, SCM, kResRegion / 256, 4, EPI, 4, WPE>), g, b, lds, s, a);
    }
}

hipError_t launch_gather_res(const KArgs& a, int mode, int rows, int sc, int waves, int re, size_t lds,
                             hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (!gath_tiles_ok(rows, sc, true) || !item_waves_ok(waves) || re < 1 || re > kResRegion || lds < 8 ||
        lds > kResLds)
        return hipErrorInvalidValue;
#define RV(R, C)                                                                                          \
    case R * 16 + C:                                                                                      \
        if (mode == GATHER_STORE) gather_res_variant<GATHER_STORE, R, C, EPI_GENERIC>(a, waves, re, lds, s); \
        else if (a.epi == EPI_ADAM_TV) gather_res_variant<GATHER_STEP, R, C, EPI_ADAM_TV>(a, waves, re, lds, s); \
        else gather_res_variant<GATHER_STEP, R, C, EPI_GENERIC>(a, waves, re, lds, s);                       \
        break
    switch (rows * 16 + sc) {
        RV(2, 1); RV(2, 2); RV(2, 4); RV(2, 8);
        RV(4, 1); RV(4, 2); RV(4, 4); RV(4, 8);
        default: return hipErrorInvalidValue;
    }
#undef RV
    return hipGetLastError();
}

hipError_t launch_gather_lists(const KArgs& a, int mode, const StageLists& L, hipStream_t s) {
    return L.tiles.gath_res
               ? launch_gather_res(a, mode, L.tiles.gath_rows, L.tiles.gath_sc, L.tiles.gath_w, L.re_gath, L.lds_res, s)
               : launch_gather(a, mode, L.tiles.gath_rows, L.tiles.gath_sc, L.tiles.gath_w, L.re_gath, s);
}

hipError_t launch_gather(const KArgs& a, int mode, int rows, int sc, int waves, int re, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (!gath_tiles_ok(rows, sc) || !item_waves_ok(waves) || re < 1 || re > kStageMax * kThreads)
        return hipErrorInvalidValue;
    return mode == GATHER_STEP ? gather_mode<GATHER_STEP>(a, rows, sc, waves, re, s)
                               : gather_mode<GATHER_STORE>(a, rows, sc, waves, re, s);
}

}  // namespace vp
