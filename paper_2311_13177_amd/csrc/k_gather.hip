// Adjoint of the projection as a gather, fused with the regulariser gradient and the
// optimiser update (Sections 4.2 and 4.3): the phased gather and the separate update pass.

#include "update.h"

namespace vp {

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
            if (a.epi == EPI_ADAM_TV && a.stream)                    \
                gather_variant<MODE, R, C, EPI_ADAM_TV | EPI_STREAM>(a, waves, re, s); \
            else if (a.epi == EPI_ADAM_TV)                           \
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
#define UV(SC)                                                                                         \
    case SC:                                                                                           \
        if (fast && a.stream) hipLaunchKernelGGL((k_update<SC, EPI_ADAM_TV | EPI_STREAM>), g, b, 0, s, a); \
        else if (fast) hipLaunchKernelGGL((k_update<SC, EPI_ADAM_TV>), g, b, 0, s, a);                 \
        else hipLaunchKernelGGL((k_update<SC, EPI_GENERIC>), g, b, 0, s, a);                           \
        break
    switch (sc) {
        UV(2); UV(4); UV(8);
        default: return hipErrorInvalidValue;
    }
#undef UV
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
