// Adjoint of the projection as a gather, fused with the regulariser gradient and the
// optimiser update (Sections 4.2 and 4.3).

#include "kcommon.h"

namespace vp {

// Whole-wave lane shifts by one (DPP wave_shr / wave_shl): lane i receives lane i - 1
// (shfl_up1) or lane i + 1 (shfl_down1); the lane without a source reads zero.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float2 shfl_up1(float2 v) { return make_float2(dpp_f<0x138>(v.x), dpp_f<0x138>(v.y)); }
__device__ __forceinline__ float2 shfl_down1(float2 v) { return make_float2(dpp_f<0x130>(v.x), dpp_f<0x130>(v.y)); }

// ------------------------------------------------------------------ optimiser update of a column

struct UpdateArgs {
    int n, S, T, kt, y0, x0, lane, sw, ns, opt;
    float lr, beta1, beta2, c1, c2, aeps, tv_w, l1_w, eps2, inv_bc2s, step_size;
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
    const int n = u.n, S = u.S;
    const int nn = n * n;
    const int kvol = S * nn;  // elements of one knot's volume (at most 2^26)
    const size_t kbase = (size_t)u.kt * kvol;
    const int x = u.x0 + u.lane, xc = min(x, n - 1);
    const float eps2 = u.eps2;
    const bool tv = EPI == EPI_ADAM_TV || u.tv_w != 0.f;
    const bool adam = EPI == EPI_ADAM_TV || u.opt == VP_OPT_ADAM;
    const bool l1 = EPI != EPI_ADAM_TV && u.l1_w != 0.f;
    const float2 nzero = make_float2(-0.f, -0.f);
    const float2 zero = make_float2(0.f, 0.f);
    // Buffers over this knot's volume in each array (and the neighbouring knots' volumes):
    // a bin's offset is scalar (soffset) and a row's lane offset a fixed 32-bit voffset,
    // so no load or store needs 64-bit address arithmetic. Rows outside the grid read
    // zero through an out-of-range voffset.
    const __amdgpu_buffer_rsrc_t rV = plane_rsrc(Vin + kbase, kvol);
    const __amdgpu_buffer_rsrc_t rP = plane_rsrc(u.kt > 0 ? Vin + kbase - kvol : Vin, u.kt > 0 ? kvol : 0);
    const __amdgpu_buffer_rsrc_t rN = plane_rsrc(u.kt + 1 < u.T ? Vin + kbase + kvol : Vin, u.kt + 1 < u.T ? kvol : 0);
    const __amdgpu_buffer_rsrc_t rO = plane_rsrc(Vout + kbase, kvol);
    const __amdgpu_buffer_rsrc_t rM = plane_rsrc(adam ? Mm + kbase : Vin, adam ? kvol : 0);
    const __amdgpu_buffer_rsrc_t rW = plane_rsrc(adam ? Mv + kbase : Vin, adam ? kvol : 0);
    auto ld = [](__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    };
    auto st = [](__amdgpu_buffer_rsrc_t r, float2 v, int voff, int soff) {
        using v2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2, v), r, voff, soff, 0);
    };
    int rb[WR];  // byte offsets of the window rows y0 - 1 .. y0 + PPT (out of range outside the grid)
#pragma unroll
    for (int r = 0; r < WR; ++r) {
        const int y = u.y0 - 1 + r;
        rb[r] = (y >= 0 && y < n) ? (y * n + xc) * (int)sizeof(float2) : kBufferOut;
    }
    auto load_plane = [&](int s, float2 (&w)[WR]) {
        if (s >= 0 && s < S) {
#pragma unroll
            for (int k = 0; k < WR; ++k) w[k] = ld(rV, rb[k], s * nn * (int)sizeof(float2));
        } else {
#pragma unroll
            for (int k = 0; k < WR; ++k) w[k] = zero;
        }
    };
    // x halos of the tile's rows: lane i < PPT reads column x0 - 1 of row y0 + i and lane
    // 32 + i column x0 + 64 (out of range, hence zero, past the grid's border or its last
    // row); lanes 0 and 63 take them by readlane, so one load per bin serves every row
    int hb = kBufferOut;
    if (u.lane < PPT) {
        const int y = u.y0 + u.lane;
        if (y < n && u.x0 > 0) hb = (y * n + u.x0 - 1) * (int)sizeof(float2);
    } else if (u.lane >= 32 && u.lane < 32 + PPT) {
        const int y = u.y0 + u.lane - 32;
        if (y < n && u.x0 + 64 < n) hb = (y * n + u.x0 + 64) * (int)sizeof(float2);
    }
    auto lane_val = [](float2 v, int l) {
        return make_float2(__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.x), l)),
                           __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.y), l)));
    };
    if (u.ns <= 0) return;
    // win[k]: rows of bin sw - 1 + k; the loop over bins is unrolled, so bin q reads
    // win[q], win[q + 1], win[q + 2] in place (no register copies between bins)
    float2 win[SCM + 2][WR];
    load_plane(u.sw - 1, win[0]);
    load_plane(u.sw, win[1]);
    load_plane(u.sw + 1, win[2]);
    float2 ws[SCM + 1][PPT];  // ws[k]: weights of the differences between bins sw - 1 + k and sw + k
#pragma unroll
    for (int i = 0; i < PPT; ++i) ws[0][i] = (tv && u.sw > 0) ? charb_w(csub(win[1][i + 1], win[0][i + 1]), eps2) : zero;
#pragma unroll
    for (int q = 0; q < SCM; ++q) {
        if (q < u.ns) {
            const int s = u.sw + q;
            if (q > 0) load_plane(s + 1, win[q + 2]);
            const float2(&cv)[WR] = win[q + 1];
            const float2(&nv)[WR] = win[q + 2];
            const int so = s * nn * (int)sizeof(float2);
            // moments, time neighbours and x halos first, so their loads overlap the arithmetic
            const float2 hv = ld(rV, hb, so);
            float2 mm[PPT], vv[PPT], tp[PPT], tn[PPT];
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                mm[i] = vv[i] = tp[i] = tn[i] = zero;
                if (adam) {
                    mm[i] = PRE ? pm[q][i] : ld(rM, rb[i + 1], so);
                    vv[i] = PRE ? pv[q][i] : ld(rW, rb[i + 1], so);
                }
                if (tv && u.kt > 0) tp[i] = ld(rP, rb[i + 1], so);
                if (tv && u.kt + 1 < u.T) tn[i] = ld(rN, rb[i + 1], so);
            }
            float2 wy[PPT + 1];
#pragma unroll
            for (int r = 0; r <= PPT; ++r) wy[r] = tv ? charb_w(csub(cv[r + 1], cv[r]), eps2) : zero;
#pragma unroll
            for (int i = 0; i < PPT; ++i)
                ws[q + 1][i] = (tv && s + 1 < S) ? charb_w(csub(nv[i + 1], cv[i + 1]), eps2) : zero;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int y = u.y0 + i;
                if (y < n) {
                    const int vo = rb[i + 1];
                    const float2 v0 = cv[i + 1];
                    float2 left = shfl_up1(v0), right = shfl_down1(v0);
                    const float2 hl = lane_val(hv, i), hr = lane_val(hv, 32 + i);
                    if (u.lane == 0) left = hl;
                    if (u.lane == 63) right = hr;
                    float2 g = nzero;
                    if (tv) {
                        if (u.kt > 0) g = cadd(g, charb_w(csub(v0, tp[i]), eps2));
                        if (u.kt + 1 < u.T) g = csub(g, charb_w(csub(tn[i], v0), eps2));
                        g = cadd(g, ws[q][i]);
                        g = csub(g, ws[q + 1][i]);
                        if (y > 0) g = cadd(g, wy[i]);
                        if (y + 1 < n) g = csub(g, wy[i + 1]);
                        if (x > 0) g = cadd(g, charb_w(csub(v0, left), eps2));
                        if (x + 1 < n) g = csub(g, charb_w(csub(right, v0), eps2));
                        g = cscale(g, u.tv_w);
                    }
                    if (l1) g = cfma(u.l1_w, charb_w(v0, eps2), g);
                    const float2 gr = cadd(acc[q][i], g);
                    if (x < n) {
                        float2 nvx;
                        if (adam) {
                            float2 m = mm[i], v = vv[i];
                            const float c1 = u.c1, c2 = u.c2;
                            m.x = __builtin_fmaf(u.beta1, m.x, c1 * gr.x);
                            m.y = __builtin_fmaf(u.beta1, m.y, c1 * gr.y);
                            v.x = __builtin_fmaf(u.beta2, v.x, (c2 * gr.x) * gr.x);
                            v.y = __builtin_fmaf(u.beta2, v.y, (c2 * gr.y) * gr.y);
                            st(rM, m, vo, so);
                            st(rW, v, vo, so);
                            // hardware square root and reciprocal (about 1 ulp each)
                            const float dx = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.x), u.inv_bc2s, u.aeps);
                            const float dy = __builtin_fmaf(__builtin_amdgcn_sqrtf(v.y), u.inv_bc2s, u.aeps);
                            nvx = make_float2(__builtin_fmaf(-u.step_size, m.x * __builtin_amdgcn_rcpf(dx), v0.x),
                                              __builtin_fmaf(-u.step_size, m.y * __builtin_amdgcn_rcpf(dy), v0.y));
                        } else {
                            nvx = make_float2(__builtin_fmaf(-u.lr, gr.x, v0.x), __builtin_fmaf(-u.lr, gr.y, v0.y));
                        }
                        st(rO, nvx, vo, so);
                    }
                }
            }
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

hipError_t launch_gather(const KArgs& a, int mode, int rows, int sc, int waves, int re, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (!gath_tiles_ok(rows, sc) || !item_waves_ok(waves) || re < 1 || re > kStageMax * kThreads)
        return hipErrorInvalidValue;
    return mode == GATHER_STEP ? gather_mode<GATHER_STEP>(a, rows, sc, waves, re, s)
                               : gather_mode<GATHER_STORE>(a, rows, sc, waves, re, s);
}

}  // namespace vp
