// Sheared spectral projection (Section 4.2 "Projection").

#include "kcommon.h"

namespace vp {

// ------------------------------------------------------------------ projection
//
// P_b[y][x] = sum_s sum_taps w * V_s[y + oy + (0|1)][x + ox + (0|1)]   (Section 4.2)
// Work item: (part group, tile row, tile column), tile = 64 columns x PPT rows, NW waves
// (4 or 8) sharing the staged volume regions. Part e of the group belongs to wave
// e % NW, slot e / NW. Each lane owns one column and accumulates PPT rows for each of
// its GW parts over the bins in ascending order.

template <int GW, int PPT, int SE, int P, int NW>
__global__ __launch_bounds__(64 * NW) void k_project(const KArgs a) {
    extern __shared__ float2 sm[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.snap) step_snapshot(a);
    for (int ti = xcd_item(blockIdx.x, gridDim.x); ti < a.ntasks; ti += gridDim.x) {
        const AS4 Task* tk = cst(a.tasks) + ti;
        const int slice = tk->slice;
        int* const stepp = DF(step);
        const int st = read_step(stepp);
        if (stepp && st >= DF(step_limit)) continue;
        const int n = DF(n), S = DF(S), B = DF(B), nparts = DF(nparts), sched = DF(schedule);
        const unsigned sseed = DF(sched_seed);
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
            const int e = j * NW + wave;
            act[j] = false;
            eb[j] = 0;
            ep[j] = 0;
            if (e < gne) {
                eb[j] = ent[ge0 + e].blade;
                ep[j] = ent[ge0 + e].part;
                act[j] = active_blade(sched, sseed, stepp, st, B, eb[j]);
            }
        }
        float2 acc[GW][PPT];
#pragma unroll
        for (int j = 0; j < GW; ++j)
#pragma unroll
            for (int i = 0; i < PPT; ++i) acc[j][i] = make_float2(0.f, 0.f);
        Stager<SE, P, 64 * NW> sg;
        sg.init(RH, RW, y0 + oymin, x0 + oxmin, n);
        float2 pre[P][SE];
        {
            const float2* planes[P];
#pragma unroll
            for (int p = 0; p < P; ++p) planes[p] = p < S ? V + (size_t)p * nn : nullptr;
            sg.fetch(planes, (int)nn, pre);
        }
        for (int s0 = 0, it = 0; s0 < S; s0 += P, ++it) {
            float2* buf = sm + (it & 1) * P * RE;
            sg.store(buf, pre);
            __syncthreads();
            if (s0 + P < S) {
                const float2* planes[P];
#pragma unroll
                for (int p = 0; p < P; ++p) planes[p] = s0 + P + p < S ? V + (size_t)(s0 + P + p) * nn : nullptr;
                sg.fetch(planes, (int)nn, pre);
            }
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int s = s0 + p;
                if (s < S) {
                    // the bin's taps for every part of the wave, loaded before any is used
                    // (a part slot without a part reads blade 0's entry and is skipped)
                    int tox[GW], toy[GW];
                    float tw[GW][4];
#pragma unroll
                    for (int j = 0; j < GW; ++j) {
                        const AS4 ShearEntry* sh = shear + eb[j] * S + s;
                        tox[j] = sh->ox;
                        toy[j] = sh->oy;
                        tw[j][0] = sh->w00;
                        tw[j][1] = sh->w01;
                        tw[j][2] = sh->w10;
                        tw[j][3] = sh->w11;
                    }
#pragma unroll
                    for (int j = 0; j < GW; ++j) {
                        if (act[j]) {
                            const float w00 = tw[j][0], w01 = tw[j][1], w10 = tw[j][2], w11 = tw[j][3];
                            const float2* L = buf + p * RE + (toy[j] - oymin) * RW + (tox[j] - oxmin) + lane;
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

// ------------------------------------------------------------------ launchers

static inline int grid_for(int ntasks) { return ntasks < 1 ? 1 : (ntasks > (1 << 20) ? (1 << 20) : ntasks); }

// The staging depth (planes per phase, elements per thread) follows the region size as
// for 256 threads; 512 threads need half the elements each (rounded up).
template <int GW, int PPT>
static void project_variant(const KArgs& a, int waves, int re, hipStream_t s) {
    const dim3 g(grid_for(a.ntasks)), b(64 * waves);
    const int depth = stage_depth(re);
    const size_t lds = stage_lds_bytes(re);
    if (waves == 8) {
        if (depth == 5) hipLaunchKernelGGL((k_project<GW, PPT, 3, 3, 8>), g, b, lds, s, a);
        else if (depth == 8) hipLaunchKernelGGL((k_project<GW, PPT, 4, 2, 8>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_project<GW, PPT, 8, 1, 8>), g, b, lds, s, a);
    } else {
        if (depth == 5) hipLaunchKernelGGL((k_project<GW, PPT, 5, 3, 4>), g, b, lds, s, a);
        else if (depth == 8) hipLaunchKernelGGL((k_project<GW, PPT, 8, 2, 4>), g, b, lds, s, a);
        else hipLaunchKernelGGL((k_project<GW, PPT, 16, 1, 4>), g, b, lds, s, a);
    }
}

hipError_t launch_project(const KArgs& a, int rows, int gw, int waves, int re, hipStream_t s) {
    if (a.ntasks <= 0) return hipSuccess;
    if (!proj_tiles_ok(rows, gw) || !item_waves_ok(waves) || re < 1 || re > kStageMax * kThreads)
        return hipErrorInvalidValue;
#define PV(R, G)                                          \
    case R * 16 + G:                                      \
        if constexpr (proj_tiles_ok(R, G)) project_variant<G, R>(a, waves, re, s); \
        break
    switch (rows * 16 + gw) {
        PV(1, 1); PV(1, 2); PV(1, 4); PV(1, 8);
        PV(2, 1); PV(2, 2); PV(2, 4); PV(2, 8);
        PV(4, 1); PV(4, 2); PV(4, 4);
        PV(8, 1); PV(8, 2); PV(12, 1);
        default: return hipErrorInvalidValue;
    }
#undef PV
    return hipGetLastError();
}

}  // namespace vp
