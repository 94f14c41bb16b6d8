// Adjoint of the projection as a gather with every blade part of a knot resident in
// LDS, fused with the regulariser gradient and the optimiser update (Sections 4.2 and
// 4.3).

#include "update.h"

namespace vp {

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

// ------------------------------------------------------------------ launcher

static inline int grid_for(int ntasks) { return ntasks < 1 ? 1 : (ntasks > (1 << 20) ? (1 << 20) : ntasks); }

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
        else if (a.epi == EPI_ADAM_TV && a.stream)                                                        \
            gather_res_variant<GATHER_STEP, R, C, EPI_ADAM_TV | EPI_STREAM>(a, waves, re, lds, s);          \
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

}  // namespace vp
