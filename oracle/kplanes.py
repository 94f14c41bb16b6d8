"""Plain FP64 implementation of the complex K-Planes dynamic volume model and its fit.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (Section 4.1, the K-Planes equation): the dynamic volume over
(x, y, omega, t) is six complex feature grids, one per pair of axes (xy, x-omega, xt,
y-omega, yt, omega-t), and a complex weight vector a. A sample projects its 4D
coordinate onto each grid, interpolates a feature vector bilinearly there, multiplies
the six vectors elementwise and takes the inner product with a. The feature dimension
is 8; two scales, one at the image resolution and one at half of it in x and y, are
summed. Section 4.2 projects the volume at each blade's time exactly as for the voxel
grid; Section 4.3 adds temporal smoothness and sparsity terms to the fit.

Readings where the paper is silent (each one also listed in the design notes):
  K1  Grid coordinates: integer voxel index i in [0, m) maps to u = i (R - 1) / (m - 1)
      on an axis of R nodes (end points on end points), so a full-resolution axis is
      read at its nodes; linear interpolation between nodes floor(u) (at most R - 2)
      and the next. Time tau in [0, 1] maps to u = tau (R_t - 1) the same way. The
      spectral axis has S nodes, so bins are read at nodes.
  K2  Scales: each scale has its own six grids with its own x/y resolution; omega and
      t keep S and R_t nodes at every scale; the scales' values are summed; one
      weight vector a serves all scales. The inner product is the bilinear sum
      sum_f a_f prod_c p_c,f (no conjugation).
  K3  Regularisers on the grids: Charbonnier total variation (as for the voxel grid)
      along each grid's x, y and omega axes, weight tv; temporal smoothness as the
      squared second difference along t of the three time grids, weight smooth;
      temporal sparsity as the Charbonnier modulus of (p - 1) on the time grids,
      weight sparse (time grids at 1 leave the static grids alone).
  K4  Parameters are optimised with the same Adam on (Re, Im) pairs; the gradient is
      dL/dRe + i dL/dIm, which for the holomorphic decoder is the conjugate partial
      derivative times the volume gradient.
  K5  Flat parameter layout: for each scale c in order the grids xy [R_c][R_c][F]
      (row y), x-omega [S][R_c][F], y-omega [S][R_c][F], xt [R_t][R_c][F],
      yt [R_t][R_c][F], omega-t [R_t][S][F]; then a [F]. All complex.
"""

from __future__ import annotations

import dataclasses
from typing import Sequence

import numpy as np

from .lifted import (Geometry, adam_update, blade_masks, data_loss, displacement, knot_weights,
                     project_blade, shear_transpose, _charbonnier)

PLANES = ("xy", "xs", "ys", "xt", "yt", "st")


@dataclasses.dataclass(frozen=True)
class KPConfig:
    """Feature count F, time nodes R_t and the x/y resolution of each scale (K2)."""
    features: int
    time_res: int
    spatial_res: tuple

    def plane_shapes(self, n_spec: int, r: int) -> dict:
        f, rt, s = self.features, self.time_res, n_spec
        return {"xy": (r, r, f), "xs": (s, r, f), "ys": (s, r, f),
                "xt": (rt, r, f), "yt": (rt, r, f), "st": (rt, s, f)}


def layout(n_spec: int, cfg: KPConfig):
    """Offsets and shapes of every grid in the flat parameter vector (K5) and its length."""
    out, off = [], 0
    for r in cfg.spatial_res:
        scale = {}
        for name, shp in cfg.plane_shapes(n_spec, r).items():
            scale[name] = (off, shp)
            off += int(np.prod(shp))
        out.append(scale)
    a_off = off
    return out, a_off, off + cfg.features


def unpack(params: np.ndarray, n_spec: int, cfg: KPConfig):
    scales, a_off, total = layout(n_spec, cfg)
    assert params.shape == (total,)
    grids = [{k: params[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in sc.items()} for sc in scales]
    return grids, params[a_off:a_off + cfg.features]


# ------------------------------------------------------------------ interpolation (K1)

def lerp_nodes(m: int, r: int):
    """Lower node, upper node and weight of the linear interpolation of an r-node axis at
    the m integer coordinates 0 .. m - 1 (K1)."""
    if r == 1:
        z = np.zeros(m, dtype=np.int64)
        return z, z, np.zeros(m)
    u = np.arange(m, dtype=np.float64) * (r - 1) / (m - 1) if m > 1 else np.zeros(m)
    i0 = np.minimum(np.floor(u).astype(np.int64), r - 2)
    return i0, i0 + 1, u - i0


def interp(p: np.ndarray, axis: int, nodes) -> np.ndarray:
    i0, i1, w = nodes
    shp = [1] * p.ndim
    shp[axis] = -1
    w = w.reshape(shp)
    return (1.0 - w) * np.take(p, i0, axis=axis) + w * np.take(p, i1, axis=axis)


def interp_transpose(g: np.ndarray, axis: int, nodes, r: int) -> np.ndarray:
    """The transpose of ``interp``: each sample's value added back onto its two nodes."""
    i0, i1, w = nodes
    shp = list(g.shape)
    shp[axis] = r
    out = np.zeros(shp, dtype=np.complex128)
    gm = np.moveaxis(g, axis, 0)
    om = np.moveaxis(out, axis, 0)
    wshape = (-1,) + (1,) * (gm.ndim - 1)
    np.add.at(om, i0, (1.0 - w).reshape(wshape) * gm)
    np.add.at(om, i1, w.reshape(wshape) * gm)
    return out


# ------------------------------------------------------------------ decoder (Section 4.1)

def _factors(grids: dict, n: int, r: int, rt: int, tau: float):
    """The scale's grids read at every voxel of the n x n x S grid at time tau:
    Z [n(y)][n(x)][F], X [S][n(x)][F], Y [S][n(y)][F], qx [n(x)][F], qy [n(y)][F], qs [S][F]."""
    nx = lerp_nodes(n, r)
    k, al = knot_weights(tau, rt)
    tw = [(k, 1.0 - al)] + ([(k + 1, al)] if rt > 1 else [])
    z = interp(interp(grids["xy"], 1, nx), 0, nx)
    x = interp(grids["xs"], 1, nx)
    y = interp(grids["ys"], 1, nx)
    qx = sum(w * interp(grids["xt"][j], 0, nx) for j, w in tw)
    qy = sum(w * interp(grids["yt"][j], 0, nx) for j, w in tw)
    qs = sum(w * grids["st"][j] for j, w in tw)
    return z, x, y, qx, qy, qs, nx, tw


def decode(params: np.ndarray, n: int, n_spec: int, cfg: KPConfig, tau: float) -> np.ndarray:
    """f(x, y, omega_s, tau) at every voxel: [S][n][n] (Section 4.1, K1, K2)."""
    grids, a = unpack(params.astype(np.complex128), n_spec, cfg)
    vol = np.zeros((n_spec, n, n), dtype=np.complex128)
    for g, r in zip(grids, cfg.spatial_res):
        z, x, y, qx, qy, qs, _, _ = _factors(g, n, r, cfg.time_res, tau)
        xx = x * qx[None] * qs[:, None]             # [S][x][F]
        yy = y * qy[None]                           # [S][y][F]
        prod = z[None] * xx[:, None] * yy[:, :, None]   # [S][y][x][F]
        vol += prod @ a
    return vol


def decode_adjoint(params: np.ndarray, n: int, n_spec: int, cfg: KPConfig, tau: float,
                   gvol: np.ndarray) -> np.ndarray:
    """Gradient with respect to the flat parameters of a real loss whose gradient with
    respect to decode(params, tau) is gvol (K4): each factor's gradient is the sum of
    gvol times the conjugate of the other factors, and interpolation transposes."""
    pc = params.astype(np.complex128)
    grids, a = unpack(pc, n_spec, cfg)
    scales, a_off, total = layout(n_spec, cfg)
    out = np.zeros(total, dtype=np.complex128)
    gv = gvol.astype(np.complex128)
    for g, r, sc in zip(grids, cfg.spatial_res, scales):
        z, x, y, qx, qy, qs, nx, tw = _factors(g, n, r, cfg.time_res, tau)
        xx = x * qx[None] * qs[:, None]
        yy = y * qy[None]
        G = gv[..., None]                                            # [S][y][x][1]
        g_z = np.sum(np.conj(a * xx[:, None] * yy[:, :, None]) * G, axis=0)          # [y][x][F]
        g_xx = np.sum(np.conj(a * z[None] * yy[:, :, None]) * G, axis=1)             # [S][x][F]
        g_yy = np.sum(np.conj(a * z[None] * xx[:, None]) * G, axis=2)                # [S][y][F]
        out[a_off:] += np.sum(np.conj(z[None] * xx[:, None] * yy[:, :, None]) * G, axis=(0, 1, 2))
        g_x = np.conj(qx[None] * qs[:, None]) * g_xx
        g_qx = np.sum(np.conj(x * qs[:, None]) * g_xx, axis=0)
        g_qs = np.sum(np.conj(x * qx[None]) * g_xx, axis=1)
        g_y = np.conj(qy[None]) * g_yy
        g_qy = np.sum(np.conj(y) * g_yy, axis=0)
        grads = {
            "xy": interp_transpose(interp_transpose(g_z, 0, nx, r), 1, nx, r),
            "xs": interp_transpose(g_x, 1, nx, r),
            "ys": interp_transpose(g_y, 1, nx, r),
            "xt": np.zeros(sc["xt"][1], dtype=np.complex128),
            "yt": np.zeros(sc["yt"][1], dtype=np.complex128),
            "st": np.zeros(sc["st"][1], dtype=np.complex128),
        }
        for j, w in tw:
            grads["xt"][j] += w * interp_transpose(g_qx, 0, nx, r)
            grads["yt"][j] += w * interp_transpose(g_qy, 0, nx, r)
            grads["st"][j] += w * g_qs
        for name, (o, shp) in sc.items():
            out[o:o + int(np.prod(shp))] += grads[name].ravel()
    return out


# ------------------------------------------------------------------ regularisers (K3)

_TV_AXES = {"xy": (0, 1), "xs": (0, 1), "ys": (0, 1), "xt": (1,), "yt": (1,), "st": (1,)}
_TIME = ("xt", "yt", "st")


def _tv(p: np.ndarray, axes, eps: float):
    val, grad = 0.0, np.zeros_like(p, dtype=np.complex128)
    for ax in axes:
        if p.shape[ax] < 2:
            continue
        d = np.diff(p, axis=ax)
        val += float(np.sum(_charbonnier(d, eps)))
        w = d / np.sqrt(np.abs(d) ** 2 + eps * eps)
        hi = [slice(None)] * p.ndim
        lo = [slice(None)] * p.ndim
        hi[ax] = slice(1, None)
        lo[ax] = slice(None, -1)
        grad[tuple(hi)] += w
        grad[tuple(lo)] -= w
    return val, grad


def _smooth(p: np.ndarray):
    """Sum of |p[k+1] - 2 p[k] + p[k-1]|^2 along t (axis 0) and its gradient."""
    grad = np.zeros_like(p, dtype=np.complex128)
    if p.shape[0] < 3:
        return 0.0, grad
    d2 = p[2:] - 2.0 * p[1:-1] + p[:-2]
    grad[2:] += 2.0 * d2
    grad[1:-1] -= 4.0 * d2
    grad[:-2] += 2.0 * d2
    return float(np.sum(np.abs(d2) ** 2)), grad


def regulariser(params: np.ndarray, n_spec: int, cfg: KPConfig, tv: float, smooth: float, sparse: float,
                eps: float):
    """Value and gradient of the grid regularisers (Section 4.3, K3)."""
    pc = params.astype(np.complex128)
    grids, _ = unpack(pc, n_spec, cfg)
    scales, _, total = layout(n_spec, cfg)
    val, out = 0.0, np.zeros(total, dtype=np.complex128)
    for g, sc in zip(grids, scales):
        for name, (o, shp) in sc.items():
            p = g[name]
            gr = np.zeros(shp, dtype=np.complex128)
            if tv != 0.0:
                v, d = _tv(p, _TV_AXES[name], eps)
                val += tv * v
                gr += tv * d
            if name in _TIME and smooth != 0.0:
                v, d = _smooth(p)
                val += smooth * v
                gr += smooth * d
            if name in _TIME and sparse != 0.0:
                q = p - 1.0
                val += sparse * float(np.sum(_charbonnier(q, eps)))
                gr += sparse * q / np.sqrt(np.abs(q) ** 2 + eps * eps)
            out[o:o + int(np.prod(shp))] += gr.ravel()
    return val, out


# ------------------------------------------------------------------ objective and fit

def objective_and_gradient(params: np.ndarray, geom: Geometry, y: np.ndarray, cfg: KPConfig,
                           tv: float = 0.0, smooth: float = 0.0, sparse: float = 0.0, eps: float = 1e-3,
                           blades: Sequence[int] | None = None):
    """Data term 0.5 sum_b |M_b DFT2(P_b f(., tau_b)) - M_b y_b|^2 plus the regularisers, its
    gradient with respect to the flat parameters, and the data term alone."""
    n, S = geom.n, geom.n_spec
    masks = blade_masks(geom)
    total, grad = 0.0, np.zeros_like(params, dtype=np.complex128)
    for b in (range(geom.n_blades) if blades is None else blades):
        tau = geom.tau(b)
        vol = decode(params, n, S, cfg, tau)
        k = masks[b] * np.fft.fft2(project_blade(vol, geom, b), norm="ortho")
        res = k - masks[b] * y[b].astype(np.complex128)
        total += data_loss(res)
        gimg = np.fft.ifft2(masks[b] * res, norm="ortho")
        theta = float(geom.angle_rad[b])
        gvol = np.stack([shear_transpose(gimg, displacement(theta, float(geom.spec_shift_px[s])))
                         for s in range(S)])
        grad += decode_adjoint(params, n, S, cfg, tau, gvol)
    data = total
    rv, rg = regulariser(params, S, cfg, tv, smooth, sparse, eps)
    return total + rv, grad + rg, data


def reconstruct(geom: Geometry, y: np.ndarray, cfg: KPConfig, init: np.ndarray, n_steps: int,
                tv: float = 0.0, smooth: float = 0.0, sparse: float = 0.0, eps: float = 1e-3,
                lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8,
                optimizer: str = "adam"):
    """n_steps updates of the flat parameters on the gradient over all blades (Adam or GD)."""
    p = init.astype(np.complex128).copy()
    m = np.zeros(p.shape + (2,))
    v = np.zeros(p.shape + (2,))
    for t in range(1, n_steps + 1):
        _, g, _ = objective_and_gradient(p, geom, y, cfg, tv, smooth, sparse, eps)
        if optimizer == "adam":
            p, m, v = adam_update(p, g, m, v, t, lr, beta1, beta2, adam_eps)
        else:
            p = p - lr * g
    val, _, data = objective_and_gradient(p, geom, y, cfg, tv, smooth, sparse, eps)
    return p, val, data


def render(params: np.ndarray, n: int, n_spec: int, cfg: KPConfig, times: Sequence[float], split_bin: int = -1):
    """Projection (sum over bins), water and fat images at each time (Section 4.3, Section 6)."""
    split = n_spec // 2 if split_bin < 0 else split_bin
    vols = np.stack([decode(params, n, n_spec, cfg, t) for t in times])
    return vols.sum(axis=1), vols[:, :split].sum(axis=1), vols[:, split:].sum(axis=1)
