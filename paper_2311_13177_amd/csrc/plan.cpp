// Host-only plan construction for libvp: validation, FP64 tables, launch lists.
// Nothing here touches a device, so every function is usable on a machine without one.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>

#include "plan.h"

namespace vp {

static thread_local std::string g_err;

vp_status fail(vp_status code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }

// Radix sequence of a length with no prime factor above 5 (radix-4 stages first).
static bool factor_235(int n, std::vector<int>& radices) {
    radices.clear();
    while (n % 4 == 0) { radices.push_back(4); n /= 4; }
    while (n % 2 == 0) { radices.push_back(2); n /= 2; }
    while (n % 3 == 0) { radices.push_back(3); n /= 3; }
    while (n % 5 == 0) { radices.push_back(5); n /= 5; }
    return n == 1;
}

// Signed frequency of an unshifted DFT index.
static double signed_freq(int j, int n) { return j <= (n - 1) / 2 ? (double)j : (double)(j - n); }

// Blade support (Section 4.2 "Blur", Cartesian masks of Section 7): half-open rotated
// rectangle of length n along the readout and width L across it, 1e-9 tie margin.
// Evaluated in FP64 without contraction so that every sample lands on the same side
// of a tie as a plain double-precision evaluation of the same rule.
#pragma clang fp contract(off)
static void build_mask(int n, double theta, int lines, uint8_t* out) {
    const double eps = 1e-9;
    const double c = std::cos(theta), s = std::sin(theta);
    const double rlo = -n / 2.0 - eps, rhi = n / 2.0 - eps;
    const double qlo = -lines / 2.0 - eps, qhi = lines / 2.0 - eps;
    for (int iy = 0; iy < n; ++iy) {
        const double ky = signed_freq(iy, n);
        for (int ix = 0; ix < n; ++ix) {
            const double kx = signed_freq(ix, n);
            const double r = kx * c + ky * s;
            const double q = -kx * s + ky * c;
            out[(size_t)iy * n + ix] = (r >= rlo && r < rhi && q >= qlo && q < qhi) ? 1 : 0;
        }
    }
}

// Bilinear taps of the sample at (x - dx, y - dy), d = delta * u (Sections 3 and 4.2).
static void build_shear(double theta, double delta, ShearEntry* e, float* fxo, float* fyo) {
    const double dx = delta * std::cos(theta);
    const double dy = delta * std::sin(theta);
    const double ox = std::floor(-dx), oy = std::floor(-dy);
    const double fx = -dx - ox, fy = -dy - oy;
    e->ox = (int)ox;
    e->oy = (int)oy;
    e->w00 = (float)((1.0 - fy) * (1.0 - fx));
    e->w01 = (float)((1.0 - fy) * fx);
    e->w10 = (float)(fy * (1.0 - fx));
    e->w11 = (float)(fy * fx);
    e->pad0 = e->pad1 = 0;
    *fxo = (float)fx;
    *fyo = (float)fy;
}
#pragma clang fp contract(on)

static int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Union of the shear offset extents of knot entries [e0, e1): {ox_min, ox_max, oy_min, oy_max}.
static void part_extents(const vp_plan* p, int e0, int e1, int* ext) {
    ext[0] = ext[2] = std::numeric_limits<int>::max();
    ext[1] = ext[3] = std::numeric_limits<int>::min();
    for (int e = e0; e < e1; ++e) {
        const BladeDev& bd = p->blade[p->knot_ent[e].blade];
        ext[0] = std::min(ext[0], bd.ox_min); ext[1] = std::max(ext[1], bd.ox_max);
        ext[2] = std::min(ext[2], bd.oy_min); ext[3] = std::max(ext[3], bd.oy_max);
    }
    if (e1 <= e0) ext[0] = ext[1] = ext[2] = ext[3] = 0;
}

// Elements of the region staged for a tile of `rows` x 64 outputs whose taps reach
// offsets [ox_min, ox_max + 1] x [oy_min, oy_max + 1].
static int region(int rows, int ox_min, int ox_max, int oy_min, int oy_max) {
    return (rows + oy_max - oy_min + 1) * (kTileW + ox_max - ox_min + 1);
}

// Work items of one tile shape. Projection items are ordered tile-major so that the
// groups of one tile (which read the same volume region) run side by side; gather items
// are ordered tile-major, then knot, then bin chunk, so that the items sharing a tile's
// blade regions and its neighbouring knots run side by side (see xcd_item).
static vp_status build_layout(const vp_plan* p, const Tiles& t, Layout* L) {
    if (!proj_tiles_ok(t.proj_rows, t.proj_gw) || !gath_tiles_ok(t.gath_rows, t.gath_sc, t.gath_res == 1) || !upd_tiles_ok(t.upd_sc) ||
        !item_waves_ok(t.gath_w) || !item_waves_ok(t.proj_w) || (t.gath_res != 0 && t.gath_res != 1) ||
        (t.gath_res && t.upd_sc))
        return fail(VP_ERR_UNSUPPORTED, "tile shape (%d, %d, %d, %d, %d, %d, %d, %d) is not compiled", t.proj_rows,
                    t.proj_gw, t.gath_rows, t.gath_sc, t.upd_sc, t.gath_w, t.proj_w, t.gath_res);
    const int n = p->n, S = p->S, T = p->T;
    L->tiles = t;
    L->groups.clear();
    L->t_proj.clear();
    L->t_gath.clear();
    L->t_upd.clear();
    const int group_parts = t.proj_w * t.proj_gw;
    for (int kt = 0; kt < T; ++kt) {
        for (int e0 = p->knot_ptr[kt]; e0 < p->knot_ptr[kt + 1]; e0 += group_parts) {
            ProjGroup gr{};
            gr.knot = kt;
            gr.e0 = e0;
            gr.ne = std::min(group_parts, p->knot_ptr[kt + 1] - e0);
            int ext[4];
            part_extents(p, e0, e0 + gr.ne, ext);
            gr.ox_min = ext[0]; gr.ox_max = ext[1]; gr.oy_min = ext[2]; gr.oy_max = ext[3];
            L->groups.push_back(gr);
        }
    }
    L->re_proj = 1;
    for (const ProjGroup& gr : L->groups)
        L->re_proj = std::max(L->re_proj, region(t.proj_rows, gr.ox_min, gr.ox_max, gr.oy_min, gr.oy_max));
    L->re_gath = 1;
    for (const KnotInfo& ki : p->knots)
        L->re_gath = std::max(L->re_gath, region(t.gath_rows, ki.ox_min, ki.ox_max, ki.oy_min, ki.oy_max));
    if (L->re_proj > kStageMax * kThreads || L->re_gath > kStageMax * kThreads)
        return fail(VP_ERR_UNSUPPORTED, "tile shape (%d, %d, %d, %d): staged region exceeds the LDS staging",
                    t.proj_rows, t.proj_gw, t.gath_rows, t.gath_sc);
    L->lds_res = 0;
    if (t.gath_res) {
        // every part of a knot resident at once: part j of knot kt at [j * region, (j + 1) * region)
        for (int kt = 0; kt < T; ++kt) {
            const KnotInfo& ki = p->knots[kt];
            const int np = p->knot_ptr[kt + 1] - p->knot_ptr[kt];
            const int re = region(t.gath_rows, ki.ox_min, ki.ox_max, ki.oy_min, ki.oy_max);
            if (np > kResMaxParts || re > kResRegion)
                return fail(VP_ERR_UNSUPPORTED, "resident gather: knot %d has %d parts of %d elements", kt, np, re);
            L->lds_res = std::max(L->lds_res, (size_t)np * (size_t)re * sizeof(float2));
        }
        if (L->lds_res > kResLds)
            return fail(VP_ERR_UNSUPPORTED, "resident gather: %zu bytes of LDS", L->lds_res);
        L->lds_res = std::max<size_t>(L->lds_res, 8);
    }
    const int txn = ceil_div(n, kTileW);
    const int typ = ceil_div(n, t.proj_rows), tyg = ceil_div(n, t.gath_rows);
    // group-major (knot-major): the tiles of one knot's group in row order, so the items
    // an XCD runs at once are vertically and horizontally adjacent tiles of one knot,
    // whose staged halos overlap in its L2 (no two knots share a staged region)
    for (int gi = 0; gi < (int)L->groups.size(); ++gi)
        for (int ty = 0; ty < typ; ++ty)
            for (int tx = 0; tx < txn; ++tx) L->t_proj.push_back(Task{0, gi, ty, tx});
    const int nch = ceil_div(S, t.gath_w * t.gath_sc);
    if (!t.gath_res) {
        for (int ty = 0; ty < tyg; ++ty)
            for (int tx = 0; tx < txn; ++tx)
                for (int kt = 0; kt < T; ++kt)
                    for (int ch = 0; ch < nch; ++ch) L->t_gath.push_back(Task{0, kt, ty * txn + tx, ch});
    } else {
        // Resident-parts items walk their bins in step from the start, so the items that
        // re-read each other's rows should start together: bands of tile rows, and within
        // a band knot by knot, put the tiles above and below (y halos) a few items apart
        // and the neighbouring knots (the time differences) one band-knot apart, instead
        // of the y neighbours a whole row of knots apart.
        const int band = std::max(1, std::min(tyg, ceil_div(16, txn * nch)));
        for (int ty0 = 0; ty0 < tyg; ty0 += band)
            for (int kt = 0; kt < T; ++kt)
                for (int ty = ty0; ty < std::min(tyg, ty0 + band); ++ty)
                    for (int tx = 0; tx < txn; ++tx)
                        for (int ch = 0; ch < nch; ++ch) L->t_gath.push_back(Task{0, kt, ty * txn + tx, ch});
    }
    if (t.upd_sc) {
        const int nuc = ceil_div(S, t.upd_sc), tyu = ceil_div(n, 4);
        for (int ty = 0; ty < tyu; ++ty)
            for (int tx = 0; tx < txn; ++tx)
                for (int kt = 0; kt < T; ++kt)
                    for (int ch = 0; ch < nuc; ++ch) L->t_upd.push_back(Task{0, kt, ty * txn + tx, ch});
    }
    return VP_OK;
}

static int pow2_ceil(int v) {
    int r = 1;
    while (r < v) r <<= 1;
    return r;
}

Tiles heuristic_tiles(const vp_plan* p) {
    // Eight-wave items over tall tiles, the shapes the tuner mostly picks on this device:
    // a projection item projects 8 * proj_gw parts of one knot over 8 rows (4 below n =
    // 192); a gather item covers 8 * gath_sc bins (all of S up to 64) over 4 rows, with
    // every part of its knot resident in LDS (the plan falls back to parts staged a few at
    // a time where they do not fit).
    Tiles t;
    t.proj_w = 8;
    t.proj_rows = p->n >= 192 ? 8 : 4;
    t.proj_gw = p->max_knot_parts > 8 ? 2 : 1;
    t.gath_w = 8;
    t.gath_rows = 4;
    t.gath_sc = std::min(8, pow2_ceil(ceil_div(p->S, 8)));
    t.gath_res = 1;
    return t;
}

vp_status plan_layout(const vp_plan* p, const Tiles& t, const Layout** out) {
    std::lock_guard<std::mutex> lk(p->mu);
    auto it = p->layouts.find(t.key());
    if (it != p->layouts.end()) {
        *out = it->second.get();
        return VP_OK;
    }
    std::unique_ptr<Layout> L(new (std::nothrow) Layout());
    if (!L) return fail(VP_ERR_NOMEM, "layout: out of host memory");
    try {
        const vp_status st = build_layout(p, t, L.get());
        if (st != VP_OK) return st;
    } catch (const std::bad_alloc&) {
        return fail(VP_ERR_NOMEM, "layout: out of host memory");
    }
    *out = L.get();
    p->layouts.emplace(t.key(), std::move(L));
    return VP_OK;
}

}  // namespace vp

using namespace vp;

extern "C" const char* vp_last_error(void) { return vp::g_err.c_str(); }

extern "C" const char* vp_status_string(vp_status s) {
    switch (s) {
        case VP_OK: return "ok";
        case VP_ERR_ARG: return "invalid argument";
        case VP_ERR_UNSUPPORTED: return "unsupported problem";
        case VP_ERR_DEVICE: return "device error";
        case VP_ERR_NONFINITE: return "non-finite value";
        case VP_ERR_BUDGET: return "request exceeds the memory budget";
        case VP_ERR_NOMEM: return "out of memory";
        case VP_ERR_TIMEOUT: return "timed out";
        case VP_ERR_CANCELLED: return "cancelled";
        case VP_ERR_NOT_FOUND: return "not found";
        case VP_ERR_STATE: return "invalid state";
        default: return "unknown status";
    }
}

extern "C" vp_status vp_options_default(vp_options* o) {
    if (!o) return fail(VP_ERR_ARG, "vp_options_default: NULL options");
    o->tv_weight = 1e-3f;
    o->l1_weight = 0.0f;
    o->tv_eps = 1e-3f;
    o->n_steps = 200;
    o->optimizer = VP_OPT_ADAM;
    o->lr = 1e-2f;
    o->beta1 = 0.9f;
    o->beta2 = 0.999f;
    o->adam_eps = 1e-8f;
    o->schedule = VP_SCHED_ALL_BLADES;
    o->split_bin = -1;
    o->device = 0;
    o->tiles = vp_tiles{0, 0, 0, 0, 0, 0, 0, 0};
    o->autotune = 0;
    o->seed = 0;
    o->data_weight = 1.0f;
    return VP_OK;
}

namespace vp {
// per_blade: every blade gets a knot of its own (knot b, weight 1); n_time must be B.
static vp_status plan_create(const vp_geometry* g, bool per_blade, vp_plan** out);
}  // namespace vp

extern "C" vp_status vp_plan_create(const vp_geometry* g, vp_plan** out) {
    clear_error();
    return vp::plan_create(g, false, out);
}

namespace vp {

vp_status plan_per_blade(const vp_plan* p, const vp_plan** out) {
    std::lock_guard<std::mutex> lk(p->mu_derived);
    if (!p->per_blade) {
        std::vector<double> times(p->B, 0.0);
        const vp_geometry g{p->n, p->S, p->B, p->B, p->angle.data(), p->lines.data(),
                            p->B > 1 ? times.data() : nullptr, p->shift.data()};
        vp_plan* q = nullptr;
        const vp_status st = plan_create(&g, true, &q);
        if (st != VP_OK) return st;
        p->per_blade.reset(q);
    }
    *out = p->per_blade.get();
    return VP_OK;
}

// Modified Bessel function I0 by its power series (converges for the arguments used).
static double bessel_i0(double x) {
    double sum = 1.0, term = 1.0;
    const double q = 0.25 * x * x;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * k);
        sum += term;
        if (term < 1e-17 * sum) break;
    }
    return sum;
}

vp_status plan_nu(const vp_plan* p, const NuHost** host, const vp_plan** over) {
    std::lock_guard<std::mutex> lk(p->mu_derived);
    const int n = p->n, B = p->B, M = kNuSigma * n;
    if (M > kMaxN) return fail(VP_ERR_UNSUPPORTED, "blade sampling: 2n = %d above %d", M, kMaxN);
    if (!p->over) {
        const std::vector<double> zero(1, 0.0);
        std::vector<int> lines(p->lines);
        const vp_geometry g{M, 1, 1, B, p->angle.data(), lines.data(), nullptr, zero.data()};
        vp_plan* q = nullptr;
        const vp_status st = plan_create(&g, false, &q);
        if (st != VP_OK) return st;
        p->over.reset(q);
    }
    if (!p->nu_host) {
        std::unique_ptr<NuHost> h(new (std::nothrow) NuHost());
        if (!h) return fail(VP_ERR_NOMEM, "blade sampling: out of host memory");
        const double W = kNuWidth, sig = kNuSigma;
        const double beta = M_PI * std::sqrt((W / sig) * (W / sig) * (sig - 0.5) * (sig - 0.5) - 0.8);
        h->lines = p->lines;
        h->lmax = *std::max_element(p->lines.begin(), p->lines.end());
        h->cs.resize(B);
        h->ph.assign((size_t)B * h->lmax * n, make_float2(0.f, 0.f));
        const double half = (double)(2 * (n / 2)) / n;
        double kmax = 0.0;
        for (int b = 0; b < B; ++b) {
            const double c = std::cos(p->angle[b]), s = std::sin(p->angle[b]);
            h->cs[b] = make_double2(c, s);
            for (int l = 0; l < p->lines[b]; ++l)
                for (int j = 0; j < n; ++j) {
                    const double r = j - 0.5 * n, q = l - 0.5 * p->lines[b];
                    const double kx = r * c - q * s, ky = r * s + q * c;
                    const size_t i = ((size_t)b * h->lmax + l) * n + j;
                    const double a = -M_PI * (kx + ky) * half;
                    h->ph[i] = make_float2((float)(std::cos(a) / n), (float)(std::sin(a) / n));
                    kmax = std::max(kmax, std::max(std::fabs(sig * kx), std::fabs(sig * ky)));
                }
        }
        h->kmax = (float)(kmax + 1.0);
        // 1 / (kernel transform) at the centred index x - floor(n/2): W sinh(z)/z, z^2 =
        // beta^2 - (pi W x / M)^2
        h->dea.resize(n);
        for (int x = 0; x < n; ++x) {
            const double w = M_PI * W * (double)(x - n / 2) / M;
            const double z2 = beta * beta - w * w, z = std::sqrt(std::fabs(z2));
            const double c = z == 0.0 ? W : (z2 > 0 ? W * std::sinh(z) / z : W * std::sin(z) / z);
            h->dea[x] = (float)(1.0 / c);
        }
        h->kb.resize(kNuTable + 1);
        for (int i = 0; i <= kNuTable; ++i) {
            const double t = (double)i / kNuTable;  // u / (W / 2)
            h->kb[i] = (float)bessel_i0(beta * std::sqrt(std::max(0.0, 1.0 - t * t)));
        }
        // the centred image occupies grid rows [0, n - n/2) and [M - n/2, M): the other
        // rows are zero before the forward row pass and unread after the inverse one
        for (const Task& tk : p->over->t_rows) {
            const int r0 = tk.b, r1 = std::min(M, r0 + fft_rows_per_item(M));
            if (r0 < n - n / 2 || r1 > M - n / 2) h->rows.push_back(tk);
        }
        p->nu_host = std::move(h);
    }
    *host = p->nu_host.get();
    *over = p->over.get();
    return VP_OK;
}

static vp_status plan_create(const vp_geometry* g, bool per_blade, vp_plan** out) {
    if (!g || !out) return fail(VP_ERR_ARG, "vp_plan_create: NULL geometry or output");
    if (g->n < 1 || g->n_spec < 1 || g->n_time < 1 || g->n_blades < 1)
        return fail(VP_ERR_ARG, "vp_plan_create: sizes must be >= 1 (n=%d S=%d T=%d B=%d)", g->n, g->n_spec,
                    g->n_time, g->n_blades);
    if (!g->angle_rad || !g->lines || !g->spec_shift_px)
        return fail(VP_ERR_ARG, "vp_plan_create: NULL angle, lines or shift array");
    if ((g->n_time == 1) != (g->blade_time == nullptr))
        return fail(VP_ERR_ARG, "vp_plan_create: blade_time must be NULL exactly when n_time == 1");
    if (per_blade && g->n_time != g->n_blades) return fail(VP_ERR_ARG, "per-blade plan: n_time must equal n_blades");
    if (g->n > kMaxN || g->n_spec > kMaxS || (!per_blade && g->n_time > kMaxT) || g->n_blades > kMaxB)
        return fail(VP_ERR_UNSUPPORTED, "vp_plan_create: size above the supported maximum (n<=%d S<=%d T<=%d B<=%d)",
                    kMaxN, kMaxS, kMaxT, kMaxB);
    std::vector<int> radices;
    if (!factor_235(g->n, radices))
        return fail(VP_ERR_UNSUPPORTED, "vp_plan_create: n=%d has a prime factor above 5", g->n);
    const int n = g->n, S = g->n_spec, T = g->n_time, B = g->n_blades;
    for (int b = 0; b < B; ++b) {
        if (!std::isfinite(g->angle_rad[b])) return fail(VP_ERR_ARG, "vp_plan_create: angle %d not finite", b);
        if (g->lines[b] < 1 || g->lines[b] > n)
            return fail(VP_ERR_ARG, "vp_plan_create: lines[%d]=%d outside [1, %d]", b, g->lines[b], n);
        if (g->blade_time) {
            const double t = g->blade_time[b];
            if (!std::isfinite(t) || t < 0.0 || t > 1.0)
                return fail(VP_ERR_ARG, "vp_plan_create: blade_time[%d] outside [0, 1]", b);
        }
    }
    for (int s = 0; s < S; ++s) {
        const double d = g->spec_shift_px[s];
        if (!std::isfinite(d)) return fail(VP_ERR_ARG, "vp_plan_create: spec_shift_px[%d] not finite", s);
        if (std::fabs(d) > kMaxShift)
            return fail(VP_ERR_UNSUPPORTED, "vp_plan_create: |spec_shift_px[%d]| = %g above %g px", s, d, kMaxShift);
    }

    std::unique_ptr<vp_plan> p(new (std::nothrow) vp_plan());
    if (!p) return fail(VP_ERR_NOMEM, "vp_plan_create: out of host memory");
    try {
        p->n = n; p->S = S; p->T = T; p->B = B;
        p->angle.assign(g->angle_rad, g->angle_rad + B);
        p->lines.assign(g->lines, g->lines + B);
        p->shift.assign(g->spec_shift_px, g->spec_shift_px + S);
        p->tau.assign(B, 0.0);
        if (g->blade_time) p->tau.assign(g->blade_time, g->blade_time + B);
        p->nstage = (int)radices.size();
        for (int i = 0; i < p->nstage; ++i) p->radix[i] = radices[i];
        p->nparts = (T > 1 && !per_blade) ? 2 : 1;

        // masks
        p->mask.resize((size_t)B * n * n);
        for (int b = 0; b < B; ++b) build_mask(n, p->angle[b], p->lines[b], &p->mask[(size_t)b * n * n]);

        // shear table and per-blade extents
        p->shear.resize((size_t)B * S);
        p->fx.resize((size_t)B * S);
        p->fy.resize((size_t)B * S);
        p->blade.resize(B);
        p->alpha.assign(B, 0.0f);
        for (int b = 0; b < B; ++b) {
            BladeDev& bd = p->blade[b];
            bd.ox_min = bd.oy_min = std::numeric_limits<int>::max();
            bd.ox_max = bd.oy_max = std::numeric_limits<int>::min();
            for (int s = 0; s < S; ++s) {
                ShearEntry& e = p->shear[(size_t)b * S + s];
                build_shear(p->angle[b], p->shift[s], &e, &p->fx[(size_t)b * S + s], &p->fy[(size_t)b * S + s]);
                bd.ox_min = std::min(bd.ox_min, e.ox); bd.ox_max = std::max(bd.ox_max, e.ox);
                bd.oy_min = std::min(bd.oy_min, e.oy); bd.oy_max = std::max(bd.oy_max, e.oy);
            }
            // knot of the blade's time (dense knots at k/(T-1), linear blend)
            // (a per-blade plan: the blade's own knot, weight 1)
            if (T == 1 || per_blade) {
                bd.knot = per_blade ? b : 0; bd.has0 = 1; bd.has1 = 0; bd.w0 = 1.0f; bd.w1 = 0.0f;
            } else {
                const double u = p->tau[b] * (T - 1);
                const int k = std::min((int)std::floor(u), T - 2);
                const double a = u - k;
                bd.knot = k;
                bd.has0 = (1.0 - a) != 0.0;
                bd.has1 = a != 0.0;
                bd.w0 = (float)(1.0 - a);
                bd.w1 = (float)a;
                p->alpha[b] = (float)a;
            }
            bd.pad = 0;
        }

        // knot entry lists, blades ascending within each knot
        p->knot_ptr.assign(T + 1, 0);
        for (int kt = 0; kt < T; ++kt) {
            p->knot_ptr[kt] = (int)p->knot_ent.size();
            for (int b = 0; b < B; ++b) {
                const BladeDev& bd = p->blade[b];
                if (bd.knot == kt && bd.has0) p->knot_ent.push_back(KnotEntry{b, 0, bd.w0, 0});
                if (T > 1 && bd.knot + 1 == kt && bd.has1) p->knot_ent.push_back(KnotEntry{b, 1, bd.w1, 0});
            }
        }
        p->knot_ptr[T] = (int)p->knot_ent.size();
        // the adjoint's taps per knot entry: bilinear weights times the entry's time
        // weight (exact product of the two rounded weights, rounded once)
        p->knot_tap.resize(p->knot_ent.size() * (size_t)S);
        for (size_t e = 0; e < p->knot_ent.size(); ++e) {
            const double w = p->knot_ent[e].weight;
            for (int s = 0; s < S; ++s) {
                ShearEntry t = p->shear[(size_t)p->knot_ent[e].blade * S + s];
                t.w00 = (float)(w * t.w00);
                t.w01 = (float)(w * t.w01);
                t.w10 = (float)(w * t.w10);
                t.w11 = (float)(w * t.w11);
                p->knot_tap[e * S + s] = t;
            }
        }

        // union of the shear extents of each knot's parts (the gather's staged halo)
        for (int kt = 0; kt < T; ++kt) {
            int ext[4];
            part_extents(p.get(), p->knot_ptr[kt], p->knot_ptr[kt + 1], ext);
            p->knots.push_back(KnotInfo{ext[0], ext[1], ext[2], ext[3]});
            p->max_knot_parts = std::max(p->max_knot_parts, p->knot_ptr[kt + 1] - p->knot_ptr[kt]);
        }

        // twiddles exp(-2 pi i j / n), FP64 then rounded
        p->tw.resize(n);
        for (int j = 0; j < n; ++j) {
            const double ang = -2.0 * M_PI * (double)j / (double)n;
            p->tw[j] = make_float2((float)std::cos(ang), (float)std::sin(ang));
        }

        // Two-row tiles hold the smallest staged regions of every shape with two rows: a
        // projection group's extents lie within its knot's, whatever the group size.
        for (const KnotInfo& ki : p->knots)
            if (region(2, ki.ox_min, ki.ox_max, ki.oy_min, ki.oy_max) > kStageMax * kThreads)
                return fail(VP_ERR_UNSUPPORTED, "vp_plan_create: shear extents exceed the staging capacity");
        // FFT LDS: data plus the twiddle table
        const int fb = fft_rows_per_item(n), cb = fft_cols_per_item(n);
        p->lds_rows = ((size_t)fb * n + n) * sizeof(float2);
        // column strip, twiddles, the strip's measurement and mask
        p->lds_cols = ((size_t)cb * n + n) * sizeof(float2) + (size_t)cb * n * (sizeof(float2) + 1);
        p->n_col_items = ceil_div(n, cb);

        // work lists of the tile-independent stages
        for (int b = 0; b < B; ++b)
            for (int r0 = 0; r0 < n; r0 += fb) p->t_rows.push_back(Task{0, b, r0, 0});
        for (int b = 0; b < B; ++b)
            for (int c = 0; c < p->n_col_items; ++c) p->t_cols.push_back(Task{0, b, c, 0});
        const uint64_t nvox = p->voxels();
        for (uint64_t i = 0; i * kVoxItem < nvox; ++i) p->t_vox.push_back(Task{0, (int)i, 0, 0});
        const int npb = ceil_div(n * n, kVoxItem);
        for (int kt = 0; kt < T; ++kt)
            for (int pb = 0; pb < npb; ++pb) p->t_render.push_back(Task{0, kt, pb, 0});
        p->base_tiles = heuristic_tiles(p.get());
        const Layout* L = nullptr;
        vp_status st = plan_layout(p.get(), p->base_tiles, &L);
        if (st != VP_OK) {
            // the knot's parts do not fit at once: stage them a few at a time
            clear_error();
            p->base_tiles.gath_res = 0;
            p->base_tiles.gath_sc = std::min(p->base_tiles.gath_sc, 16 / p->base_tiles.gath_rows);
            st = plan_layout(p.get(), p->base_tiles, &L);
        }
        if (st != VP_OK) {
            clear_error();
            p->base_tiles = Tiles{};
            st = plan_layout(p.get(), p->base_tiles, &L);
        }
        if (st != VP_OK) return st;
    } catch (const std::bad_alloc&) {
        return fail(VP_ERR_NOMEM, "vp_plan_create: out of host memory");
    }
    *out = p.release();
    return VP_OK;
}

}  // namespace vp

extern "C" vp_status vp_plan_shape(const vp_plan* p, int32_t* n, int32_t* s, int32_t* t, int32_t* b) {
    if (!p) return fail(VP_ERR_ARG, "vp_plan_shape: NULL plan");
    if (n) *n = p->n;
    if (s) *s = p->S;
    if (t) *t = p->T;
    if (b) *b = p->B;
    return VP_OK;
}

extern "C" vp_status vp_plan_mask(const vp_plan* p, int32_t b, uint8_t* out) {
    if (!p || !out) return fail(VP_ERR_ARG, "vp_plan_mask: NULL argument");
    if (b < 0 || b >= p->B) return fail(VP_ERR_ARG, "vp_plan_mask: blade %d outside [0, %d)", b, p->B);
    std::memcpy(out, &p->mask[(size_t)b * p->n * p->n], (size_t)p->n * p->n);
    return VP_OK;
}

extern "C" vp_status vp_plan_shear(const vp_plan* p, int32_t b, int32_t s, int32_t* ox, int32_t* oy, float* fx,
                                   float* fy) {
    if (!p) return fail(VP_ERR_ARG, "vp_plan_shear: NULL plan");
    if (b < 0 || b >= p->B || s < 0 || s >= p->S) return fail(VP_ERR_ARG, "vp_plan_shear: index out of range");
    const size_t i = (size_t)b * p->S + s;
    if (ox) *ox = p->shear[i].ox;
    if (oy) *oy = p->shear[i].oy;
    if (fx) *fx = p->fx[i];
    if (fy) *fy = p->fy[i];
    return VP_OK;
}

extern "C" vp_status vp_plan_knot(const vp_plan* p, int32_t b, int32_t* knot, float* alpha) {
    if (!p) return fail(VP_ERR_ARG, "vp_plan_knot: NULL plan");
    if (b < 0 || b >= p->B) return fail(VP_ERR_ARG, "vp_plan_knot: blade out of range");
    if (knot) *knot = p->blade[b].knot;
    if (alpha) *alpha = p->alpha[b];
    return VP_OK;
}

namespace vp {
uint64_t table_bytes(const vp_plan* p) {
    // the largest layout a plan can take: one-row projection tiles with one part per
    // wave and two-row gather tiles with one bin per wave (the most work items)
    const uint64_t tiles_proj = (uint64_t)p->n * ceil_div(p->n, kTileW);
    const uint64_t groups = (uint64_t)p->T + ceil_div(p->knot_ent.size(), 4);
    const uint64_t t_gath = (uint64_t)p->T * ceil_div(p->n, 2) * ceil_div(p->n, kTileW) * ceil_div(p->S, 4) +
                            (uint64_t)p->T * ceil_div(p->n, 4) * ceil_div(p->n, kTileW) * ceil_div(p->S, 2);
    return p->mask.size() + p->shear.size() * sizeof(ShearEntry) + p->blade.size() * sizeof(BladeDev) +
           p->knot_ptr.size() * sizeof(int) + p->knot_ent.size() * sizeof(KnotEntry) + p->knot_tap.size() * sizeof(ShearEntry) +
           groups * sizeof(ProjGroup) + p->knots.size() * sizeof(KnotInfo) + p->tw.size() * sizeof(float2) +
           (groups * tiles_proj + t_gath + p->t_rows.size() + p->t_cols.size() + p->t_vox.size() +
            p->t_render.size()) *
               sizeof(Task);
}

uint64_t state_bytes(const vp_plan* p, const vp_options* o) {
    const uint64_t vox = p->voxels() * sizeof(float2);
    uint64_t b = 2 * vox;                                         // volume ping-pong
    if (!o || o->optimizer == VP_OPT_ADAM) b += 2 * vox;          // Adam moments
    b += (uint64_t)p->nparts * p->blade_px() * sizeof(float2);   // blade work images
    b += p->blade_px() * sizeof(float2);                          // measurements
    b += loss_slots(p) * sizeof(float) + 256;                     // loss partials, step counter block
    b += 2 * p->t_vox.size() * sizeof(double);                    // objective partials
    b += 3 * (uint64_t)p->T * p->n * p->n * sizeof(float2);       // renders
    b += vox;                                                     // data gradient (separate update pass)
    return b;
}
}  // namespace vp

extern "C" vp_status vp_plan_device_bytes(const vp_plan* p, const vp_options* o, uint64_t* bytes) {
    if (!p || !bytes) return fail(VP_ERR_ARG, "vp_plan_device_bytes: NULL argument");
    *bytes = vp::state_bytes(p, o) + vp::table_bytes(p);
    return VP_OK;
}
