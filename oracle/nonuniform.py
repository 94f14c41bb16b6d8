"""Blade-aligned (non-Cartesian) k-space sampling of the lifted model, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's forward model masks a Cartesian DFT grid; its discussion notes that real
PROPELLER blades are sampled along blade-aligned lines and need a non-uniform DFT
instead, with everything else unchanged. Here blade b's samples sit on its own rotated
lattice, k = r u_b + q n_b with readout index r = j - n/2 (j < n) and line index
q = l - L_b/2 (l < L_b), u_b = (cos, sin), n_b = (-sin, cos); at 0 and 90 degrees they
are exactly the Cartesian mask's samples.

  * ``ndft_forward`` / ``ndft_adjoint``: the definition, y(k) = (1/n) sum_x f(x)
    exp(-2 pi i k.x / n) and its adjoint, evaluated directly.
  * ``nufft_forward`` / ``nufft_adjoint``: the gridding algorithm (Kaiser-Bessel kernel
    of width W on a grid oversampled by sigma, Beatty, Nishimura and Pauly, IEEE TMI
    2005): divide the centred image by the kernel's transform, zero-pad, FFT, and
    interpolate each sample from its W x W neighbourhood; the adjoint spreads, inverse
    FFTs and divides. It approximates the definition within a bound set by W and sigma.
  * the lifted data term with these samples and its gradient.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.special

from .lifted import (Geometry, adam_update, displacement, knot_weights, l1_grad, l1_value, project_blade,
                     random_blade, render, shear_transpose, tv_grad, tv_value, volume_at)

KB_WIDTH = 6.0
KB_SIGMA = 2.0


def blade_samples(n: int, theta: float, lines: int):
    """(kx, ky) [lines][n] of a blade's lattice (row l = line, column j = readout)."""
    r = np.arange(n, dtype=np.float64) - n / 2.0
    q = np.arange(lines, dtype=np.float64) - lines / 2.0
    c, s = math.cos(theta), math.sin(theta)
    kx = r[None, :] * c - q[:, None] * s
    ky = r[None, :] * s + q[:, None] * c
    return kx, ky


def ndft_forward(img: np.ndarray, kx: np.ndarray, ky: np.ndarray) -> np.ndarray:
    n = img.shape[-1]
    x = np.arange(n, dtype=np.float64)
    ex = np.exp(-2j * np.pi * kx[..., None] * x / n)     # [..., x]
    ey = np.exp(-2j * np.pi * ky[..., None] * x / n)     # [..., y]
    return np.einsum("...y,yx,...x->...", ey, img.astype(np.complex128), ex) / n


def ndft_adjoint(s: np.ndarray, kx: np.ndarray, ky: np.ndarray, n: int) -> np.ndarray:
    x = np.arange(n, dtype=np.float64)
    ex = np.exp(2j * np.pi * kx.reshape(-1)[:, None] * x / n)
    ey = np.exp(2j * np.pi * ky.reshape(-1)[:, None] * x / n)
    return np.einsum("m,my,mx->yx", s.astype(np.complex128).reshape(-1), ey, ex) / n


# ------------------------------------------------------------------ gridding (Kaiser-Bessel)

def kb_beta(w: float = KB_WIDTH, sigma: float = KB_SIGMA) -> float:
    return math.pi * math.sqrt((w / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb_kernel(u: np.ndarray, w: float = KB_WIDTH, sigma: float = KB_SIGMA) -> np.ndarray:
    """I0(beta sqrt(1 - (2u/W)^2)) on |u| <= W/2 (u in oversampled grid units), else 0."""
    t = 1.0 - (2.0 * np.asarray(u, dtype=np.float64) / w) ** 2
    return np.where(t >= 0.0, scipy.special.i0(kb_beta(w, sigma) * np.sqrt(np.maximum(t, 0.0))), 0.0)


def kb_transform(x: np.ndarray, m: int, w: float = KB_WIDTH, sigma: float = KB_SIGMA) -> np.ndarray:
    """integral of kb_kernel(u) exp(2 pi i u x / m) du: W sinh(z)/z, z^2 = beta^2 - (pi W x / m)^2."""
    b = kb_beta(w, sigma)
    z2 = b * b - (math.pi * w * np.asarray(x, dtype=np.float64) / m) ** 2
    z = np.sqrt(np.abs(z2))
    return np.where(z2 > 0, w * np.sinh(z) / np.where(z > 0, z, 1.0),
                    np.where(z > 0, w * np.sin(z) / np.where(z > 0, z, 1.0), w))


def _grid(n: int, sigma: float):
    m = int(round(sigma * n))
    xc = np.arange(n) - n // 2                      # centred image coordinates
    return m, xc


def nufft_forward(img: np.ndarray, kx: np.ndarray, ky: np.ndarray, w: float = KB_WIDTH,
                  sigma: float = KB_SIGMA) -> np.ndarray:
    """Gridding approximation of ``ndft_forward``."""
    n = img.shape[-1]
    m, xc = _grid(n, sigma)
    dea = kb_transform(xc, m, w, sigma)
    h = np.zeros((m, m), dtype=np.complex128)
    # centred image f[y][x] at (x - n/2, y - n/2) over the deapodisation, wrapped onto the grid
    h[np.ix_(xc % m, xc % m)] = img.astype(np.complex128) / np.outer(dea, dea)
    H = np.fft.fft2(h)
    out = np.zeros(kx.shape, dtype=np.complex128)
    half = w / 2.0
    for idx in np.ndindex(kx.shape):
        gx, gy = sigma * kx[idx], sigma * ky[idx]
        mx = np.arange(math.ceil(gx - half), math.floor(gx + half) + 1)
        my = np.arange(math.ceil(gy - half), math.floor(gy + half) + 1)
        cx, cy = kb_kernel(gx - mx, w, sigma), kb_kernel(gy - my, w, sigma)
        val = np.sum(np.outer(cy, cx) * H[np.ix_(my % m, mx % m)])
        # the image origin is the grid's centre: a phase for the shift by n/2
        out[idx] = val * np.exp(-1j * np.pi * (kx[idx] + ky[idx]) * (2 * (n // 2)) / n)
    return out / n


def nufft_adjoint(s: np.ndarray, kx: np.ndarray, ky: np.ndarray, n: int, w: float = KB_WIDTH,
                  sigma: float = KB_SIGMA) -> np.ndarray:
    """The exact adjoint of ``nufft_forward`` (spread, inverse FFT, divide)."""
    m, xc = _grid(n, sigma)
    G = np.zeros((m, m), dtype=np.complex128)
    half = w / 2.0
    for idx in np.ndindex(kx.shape):
        v = s[idx] * np.exp(1j * np.pi * (kx[idx] + ky[idx]) * (2 * (n // 2)) / n)
        gx, gy = sigma * kx[idx], sigma * ky[idx]
        mx = np.arange(math.ceil(gx - half), math.floor(gx + half) + 1)
        my = np.arange(math.ceil(gy - half), math.floor(gy + half) + 1)
        cx, cy = kb_kernel(gx - mx, w, sigma), kb_kernel(gy - my, w, sigma)
        np.add.at(G, np.ix_(my % m, mx % m), v * np.outer(cy, cx))
    g = np.fft.ifft2(G) * (m * m)            # unnormalised inverse transform
    dea = kb_transform(xc, m, w, sigma)
    return g[np.ix_(xc % m, xc % m)] / np.outer(dea, dea) / n


# ------------------------------------------------------------------ lifted data term

def forward_nu(vol: np.ndarray, geom: Geometry, exact: bool = True) -> list:
    """Blade b's samples [L_b][n] of the projected volume at its time (definition or gridding)."""
    out = []
    for b in range(geom.n_blades):
        kx, ky = blade_samples(geom.n, float(geom.angle_rad[b]), int(geom.lines[b]))
        p = project_blade(volume_at(vol, geom.tau(b)), geom, b)
        out.append(ndft_forward(p, kx, ky) if exact else nufft_forward(p, kx, ky))
    return out


def gradient_nu(vol: np.ndarray, geom: Geometry, y: list, exact: bool = True, blades=None):
    """Gradient (dL/dRe + i dL/dIm) of 0.5 sum_b |samples_b(V) - y_b|^2 and its value, over
    all blades or the listed ones."""
    n = geom.n
    grad = np.zeros((geom.n_time, geom.n_spec, n, n), dtype=np.complex128)
    total = 0.0
    for b, yb in enumerate(y):
        if blades is not None and b not in blades:
            continue
        theta = float(geom.angle_rad[b])
        kx, ky = blade_samples(n, theta, int(geom.lines[b]))
        p = project_blade(volume_at(vol, geom.tau(b)), geom, b)
        r = (ndft_forward(p, kx, ky) if exact else nufft_forward(p, kx, ky)) - yb
        total += 0.5 * float(np.sum(np.abs(r) ** 2))
        g = ndft_adjoint(r, kx, ky, n) if exact else nufft_adjoint(r, kx, ky, n)
        per_bin = np.stack([shear_transpose(g, displacement(theta, float(geom.spec_shift_px[s])))
                            for s in range(geom.n_spec)])
        if geom.n_time == 1:
            grad[0] += per_bin
        else:
            k, a = knot_weights(geom.tau(b), geom.n_time)
            grad[k] += (1.0 - a) * per_bin
            grad[k + 1] += a * per_bin
    return grad, total


def reconstruct_nu(geom: Geometry, y: list, n_steps: int, tv_weight: float = 1e-3, tv_eps: float = 1e-3,
                   l1_weight: float = 0.0, lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999,
                   adam_eps: float = 1e-8, optimizer: str = "adam", exact: bool = True,
                   data_weight: float = 1.0, split_bin: int = -1, schedule: str = "all",
                   seed: int = 0) -> dict:
    """The fit of Section 4.3 on blade-aligned samples: every step the gradient of the
    weighted data term plus TV and L1, then Adam or GD; from zero. The data term of step t
    covers all blades, or one (blade (t - 1) mod B, or the seeded random draw of step t - 1,
    as in the Cartesian fit); the final loss covers all blades."""
    vol = np.zeros((geom.n_time, geom.n_spec, geom.n, geom.n), dtype=np.complex128)
    m = np.zeros(vol.shape + (2,))
    v = np.zeros(vol.shape + (2,))

    def value(vv):
        _, d = gradient_nu(vv, geom, y, exact)
        out = data_weight * d
        if tv_weight != 0.0:
            out += tv_weight * tv_value(vv, tv_eps)
        if l1_weight != 0.0:
            out += l1_weight * l1_value(vv, tv_eps)
        return out

    for t in range(1, n_steps + 1):
        if schedule == "all":
            blades = None
        elif schedule == "cyclic":
            blades = [(t - 1) % geom.n_blades]
        else:
            blades = [random_blade(seed, t - 1, geom.n_blades)]
        g, _ = gradient_nu(vol, geom, y, exact, blades)
        g = data_weight * g
        if tv_weight != 0.0:
            g = g + tv_weight * tv_grad(vol, tv_eps)
        if l1_weight != 0.0:
            g = g + l1_weight * l1_grad(vol, tv_eps)
        if optimizer == "adam":
            vol, m, v = adam_update(vol, g, m, v, t, lr, beta1, beta2, adam_eps)
        else:
            vol = vol - lr * g
    proj, water, fat = render(vol, split_bin)
    return dict(vol=vol, proj=proj, water=water, fat=fat, final_loss=value(vol))


def simulate_samples(case) -> list:
    """Section 5's measurement on blade-aligned samples: blade b's lattice samples of the
    projected ground truth at its time (the definition), plus sigma times the case's noise
    on its first L_b rows; [L_b][n] per blade, complex128."""
    from synth.phantom import ground_truth_volume

    geom = Geometry.from_dict(case.geometry())
    out = []
    for b in range(geom.n_blades):
        w, f = case.layers_at(geom.tau(b))
        gt = ground_truth_volume(w, f, geom.n_spec)
        L = int(geom.lines[b])
        kx, ky = blade_samples(geom.n, float(geom.angle_rad[b]), L)
        out.append(ndft_forward(project_blade(gt, geom, b), kx, ky) + case.sigma * case.noise[b][:L, :])
    return out
