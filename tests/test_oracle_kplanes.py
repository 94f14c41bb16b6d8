"""Pins of the FP64 K-Planes oracle (Section 4.1) against things other than itself.

Brute-force per-voxel evaluation with scalar interpolation, exactness of linear
interpolation, adjoint identities of the interpolation, reduction to the (separately
pinned) dense knot model, central differences of the whole objective, and closed
forms of the regularisers.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle import kplanes as K


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _geom(n=10, s=3, b=3, times=(0.0, 0.45, 1.0)):
    return O.Geometry(n=n, n_spec=s, n_time=1, angle_rad=np.linspace(0.2, 2.6, b), lines=np.full(b, 4),
                      blade_time=np.asarray(times[:b], dtype=np.float64),
                      spec_shift_px=np.linspace(-1.1, 1.7, s))


def _params(rng, s, cfg, scale=1.0):
    _, _, total = K.layout(s, cfg)
    return scale * _crandn(rng, total)


# ------------------------------------------------------------------ interpolation (K1)

def test_lerp_reproduces_linear_functions_and_nodes():
    for m, r in ((9, 9), (9, 5), (12, 6), (7, 2), (5, 1)):
        nodes = K.lerp_nodes(m, r)
        p = 0.3 + 1.7 * np.arange(r, dtype=np.float64)       # linear on the nodes
        got = K.interp(p.astype(np.complex128), 0, nodes)
        want = 0.3 + 1.7 * np.arange(m) * (r - 1) / (m - 1) if r > 1 else np.full(m, 0.3)
        assert np.allclose(got, want, atol=1e-13)
        if m == r:  # full resolution reads the nodes themselves
            q = np.random.default_rng(m).standard_normal(r)
            assert np.allclose(K.interp(q, 0, nodes), q, atol=0)


def test_interp_transpose_is_the_adjoint():
    rng = np.random.default_rng(3)
    for m, r in ((10, 5), (10, 10), (7, 3)):
        nodes = K.lerp_nodes(m, r)
        p = _crandn(rng, 4, r, 2)
        g = _crandn(rng, 4, m, 2)
        lhs = np.vdot(g, K.interp(p, 1, nodes))
        rhs = np.vdot(K.interp_transpose(g, 1, nodes, r), p)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------------ decoder (Section 4.1)

def _bilerp_scalar(grid, u, v):
    """grid[row][col] at continuous (row u, column v), end-clamped lower nodes."""
    def split(c, r):
        if r == 1:
            return 0, 0, 0.0
        i = min(int(math.floor(c)), r - 2)
        return i, i + 1, c - i
    i0, i1, wu = split(u, grid.shape[0])
    j0, j1, wv = split(v, grid.shape[1])
    return ((1 - wu) * ((1 - wv) * grid[i0, j0] + wv * grid[i0, j1])
            + wu * ((1 - wv) * grid[i1, j0] + wv * grid[i1, j1]))


def test_decode_matches_a_per_voxel_brute_force():
    rng = np.random.default_rng(5)
    n, S = 6, 3
    cfg = K.KPConfig(features=3, time_res=4, spatial_res=(6, 3))
    p = _params(rng, S, cfg)
    grids, a = K.unpack(p, S, cfg)
    for tau in (0.0, 0.37, 1.0):
        got = K.decode(p, n, S, cfg, tau)
        for s in range(S):
            for yy in range(n):
                for xx in range(n):
                    val = 0.0
                    for g, r in zip(grids, cfg.spatial_res):
                        cx, cy = xx * (r - 1) / (n - 1), yy * (r - 1) / (n - 1)
                        ct = tau * (cfg.time_res - 1)
                        for f in range(cfg.features):
                            prod = (_bilerp_scalar(g["xy"][:, :, f], cy, cx)
                                    * _bilerp_scalar(g["xs"][:, :, f], s, cx)
                                    * _bilerp_scalar(g["ys"][:, :, f], s, cy)
                                    * _bilerp_scalar(g["xt"][:, :, f], ct, cx)
                                    * _bilerp_scalar(g["yt"][:, :, f], ct, cy)
                                    * _bilerp_scalar(g["st"][:, :, f], ct, s))
                            val += a[f] * prod
                    assert abs(got[s, yy, xx] - val) <= 1e-12 * max(1.0, abs(val))


def test_constant_grids_decode_to_the_number_of_scales():
    n, S = 8, 2
    cfg = K.KPConfig(features=2, time_res=3, spatial_res=(8, 4))
    scales, a_off, total = K.layout(S, cfg)
    p = np.ones(total, dtype=np.complex128)
    p[a_off:] = [1.0, 0.0]
    for tau in (0.0, 0.6):
        assert np.allclose(K.decode(p, n, S, cfg, tau), 2.0, atol=1e-14)


def test_spectral_time_grid_alone_is_the_dense_knot_model():
    # F = 1, a = 1, every grid 1 except omega-t: f(x, y, s, tau) is the linear blend in
    # time of st[k][s], i.e. the dense knot model with knots V[k][s] = st[k][s]; objective
    # and gradient follow the (separately pinned) dense model's
    rng = np.random.default_rng(7)
    n, S, Rt = 10, 3, 3
    geom = _geom(n=n, s=S)
    cfg = K.KPConfig(features=1, time_res=Rt, spatial_res=(n,))
    scales, a_off, total = K.layout(S, cfg)
    p = np.ones(total, dtype=np.complex128)
    o, shp = scales[0]["st"]
    st = _crandn(rng, Rt, S)
    p[o:o + st.size] = st.ravel()
    y = O.blade_masks(geom) * _crandn(rng, geom.n_blades, n, n)
    dense = np.broadcast_to(st[:, :, None, None], (Rt, S, n, n)).astype(np.complex128)
    dgeom = O.Geometry(n=n, n_spec=S, n_time=Rt, angle_rad=geom.angle_rad, lines=geom.lines,
                       blade_time=geom.blade_time, spec_shift_px=geom.spec_shift_px)
    val, grad, data = K.objective_and_gradient(p, geom, y, cfg)
    dres = O.residual(dense, dgeom, y)
    assert math.isclose(data, O.data_loss(dres), rel_tol=1e-12)
    dgrad = O.adjoint(dres, dgeom)
    assert np.allclose(grad[o:o + st.size].reshape(Rt, S), dgrad.sum(axis=(2, 3)), rtol=1e-11, atol=1e-11)


# ------------------------------------------------------------------ gradient (K4)

@pytest.mark.parametrize("weights", [(0.0, 0.0, 0.0), (0.05, 0.3, 0.02)])
def test_gradient_central_difference(weights):
    rng = np.random.default_rng(11)
    n, S = 8, 3
    geom = _geom(n=n, s=S)
    cfg = K.KPConfig(features=2, time_res=3, spatial_res=(8, 4))
    p = _params(rng, S, cfg, 0.6)
    y = O.blade_masks(geom) * _crandn(rng, geom.n_blades, n, n)
    tv, smooth, sparse = weights
    _, g, _ = K.objective_and_gradient(p, geom, y, cfg, tv, smooth, sparse, 0.05)
    for trial in range(3):
        d = _crandn(rng, p.size)
        h = 1e-5
        fp = K.objective_and_gradient(p + h * d, geom, y, cfg, tv, smooth, sparse, 0.05)[0]
        fm = K.objective_and_gradient(p - h * d, geom, y, cfg, tv, smooth, sparse, 0.05)[0]
        fd = (fp - fm) / (2 * h)
        an = float(np.sum((np.conj(g) * d).real))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)


# ------------------------------------------------------------------ regularisers (K3)

def test_regulariser_closed_forms():
    S = 3
    cfg = K.KPConfig(features=2, time_res=4, spatial_res=(6,))
    scales, a_off, total = K.layout(S, cfg)
    # time grids linear in t: no smoothness cost; all grids constant: no TV
    p = np.zeros(total, dtype=np.complex128)
    for name, (o, shp) in scales[0].items():
        g = np.broadcast_to((0.5 - 0.25j) * np.arange(shp[0])[:, None, None], shp) if name in ("xt", "yt", "st") \
            else np.full(shp, 0.7 + 0.1j)
        p[o:o + g.size] = np.asarray(g).ravel()
    v, _ = K.regulariser(p, S, cfg, 0.0, 1.0, 0.0, 1e-3)
    assert v == 0.0
    # constant grids: TV is zero; time grids at 1: sparsity is zero
    q = np.full(total, 1.0 + 0j)
    assert K.regulariser(q, S, cfg, 1.0, 1.0, 1.0, 1e-3)[0] == 0.0
    # a single jump of height h along x of the xy grid: TV = rows * F * (sqrt(h^2+e^2) - e)
    r = np.full(total, 1.0 + 0j)
    o, shp = scales[0]["xy"]
    g = np.ones(shp, dtype=np.complex128)
    g[:, 3:, :] = 1.0 + 0.4
    r[o:o + g.size] = g.ravel()
    e = 1e-3
    assert math.isclose(K.regulariser(r, S, cfg, 1.0, 0.0, 0.0, e)[0], shp[0] * shp[2] * (math.sqrt(0.16 + e * e) - e),
                        rel_tol=1e-12)
    # a quadratic bump in time: smoothness = sum of squared second differences
    s2 = np.full(total, 1.0 + 0j)
    o, shp = scales[0]["st"]
    g = np.ones(shp, dtype=np.complex128)
    g[1] += 0.3j
    s2[o:o + g.size] = g.ravel()
    # second differences 0.3j*(-2) at k=1 and 0.3j*(1) at k=2, per (s, f)
    want = shp[1] * shp[2] * (0.6 ** 2 + 0.3 ** 2)
    assert math.isclose(K.regulariser(s2, S, cfg, 0.0, 1.0, 0.0, e)[0], want, rel_tol=1e-12)


def test_gd_descends_and_adam_first_step():
    rng = np.random.default_rng(13)
    n, S = 8, 2
    geom = _geom(n=n, s=S)
    cfg = K.KPConfig(features=2, time_res=3, spatial_res=(8, 4))
    p0 = _params(rng, S, cfg, 0.3)
    y = O.blade_masks(geom) * _crandn(rng, geom.n_blades, n, n)
    v0 = K.objective_and_gradient(p0, geom, y, cfg, 0.01, 0.01, 0.01)[0]
    p1, v1, _ = K.reconstruct(geom, y, cfg, p0, 3, 0.01, 0.01, 0.01, lr=1e-3, optimizer="gd")
    assert v1 < v0
    # Adam's first step moves every real component by lr * g / (|g| + eps)
    _, g, _ = K.objective_and_gradient(p0, geom, y, cfg)
    p2, _, _ = K.reconstruct(geom, y, cfg, p0, 1, lr=1e-2)
    step = p0 - p2
    assert np.allclose(step.real, 1e-2 * g.real / (np.abs(g.real) + 1e-8), atol=1e-12)
    assert np.allclose(step.imag, 1e-2 * g.imag / (np.abs(g.imag) + 1e-8), atol=1e-12)


def test_seeded_init_follows_the_oracle_layout():
    from synth.kplanes_init import grid_sizes, init_params

    cfg = K.KPConfig(features=4, time_res=5, spatial_res=(12, 6))
    scales, a_off, total = K.layout(3, cfg)
    sizes = grid_sizes(3, 4, 5, (12, 6))
    assert sum(sz for _, sz in sizes) == total
    p = init_params(3, 4, 5, (12, 6), seed=1)
    grids, a = K.unpack(p, 3, cfg)
    for g in grids:
        assert np.all((g["xy"].real >= 0.1) & (g["xy"].real < 0.5)) and np.all(g["xt"] == 1.0)
    assert np.all(a == 0)
