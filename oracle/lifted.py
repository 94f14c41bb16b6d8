"""Plain FP64 implementation of the lifted PROPELLER forward model, its adjoint and the fit.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes:
  * Section 3: a frequency offset on a PROPELLER blade is a linear phase along the
    blade's readout, hence a translation of the image along the readout direction.
  * Section 4.1: the static model is a complex voxel grid over (x, y, omega); the
    dynamic model adds time.
  * Section 4.2, "Projection": one ray per pixel, samples interpolated from the
    volume and summed; each blade has an in-plane angle theta and a tilt phi off
    the spectral axis, so material at spectral height omega lands shifted along
    the blade direction.
  * Section 4.2, "Blur": the projected image goes through a 2D DFT and the blade's
    k-space support mask; an inverse DFT returns it to image space.
  * Section 4.3: squared L2 data terms, total variation along the spatial and
    spectral (and, dynamic, temporal) axes, an L1 term, Adam updates, and a final
    render with phi = 0 (straight sum along the spectral axis).
  * Section 6: the baseline is a coverage-weighted average of the blades in
    k-space followed by an inverse DFT; fat and water are the lower and upper
    portions of the spectral axis.

Readings where the paper is silent (each one also listed in the design notes):
  R1  theta is the readout (long-axis) direction of the blade: u = (cos, sin) in
      (x = column, y = row); the blade's lines stack along (-sin, cos).
  R2  The caller passes the shift of each spectral bin, delta_s, in pixels along u
      (delta_s = tan(phi) * omega_s); a positive delta moves material along +u.
  R3  One sample per spectral plane (integer s), so the trilinear sample reduces to
      bilinear interpolation in-plane; unit ray weight.
  R4  Interpolation taps outside the N x N grid read zero (no wrap, no clamp).
  R5  The DFT is unitary ("ortho") with unshifted storage: index j holds the
      signed frequency j for j <= (n-1)//2 and j - n otherwise.
  R6  Blade mask: half-open rotated rectangle, length n along u and width L along
      the line direction, with a 1e-9 tie margin.
  R7  Under a unitary DFT the k-space and image-space squared errors of the same
      masked residual are equal (Parseval), so the data term is 0.5 * sum |R|^2.
  R8  TV is anisotropic Charbonnier on the complex modulus with forward
      differences only where the neighbour exists, summed over every axis of the
      [T][S][n][n] volume (the t axis is empty when T = 1); L1 is the Charbonnier
      modulus. Both use the same epsilon.
  R9  Adam with torch's defaults acts on (Re, Im) as independent real parameters;
      t counts from 1; the volume starts at zero. GD is an option.
  R10 A step is one update on the gradient summed over all blades; the paper's
      one-blade-per-iteration schedule is an option, either in turn ("cyclic", blade
      (t-1) mod B) or drawn at random ("random": blade splitmix64(seed * 2^32 + t - 1)
      mod B, the SplitMix64 generator of Steele, Lea and Flood, 2014).
  R11 Dynamic: a dense grid of T time knots at k/(T-1); a blade at time tau sees
      (1-a) V[k] + a V[k+1] with k = floor(tau (T-1)) clamped to T-2, a = tau (T-1) - k.
  R12 Fat/water split at bin S/2 by default; water = bins below it, fat = the rest.
  R16 The image-space and k-space squared errors (Section 4.3) are the same number
      under a unitary DFT (R7), so their weighted sum is data_weight * 0.5 * sum |R|^2
      with data_weight = w_image + w_kspace (1 by default).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

MASK_EPS = 1e-9


# --------------------------------------------------------------------------- geometry

@dataclasses.dataclass
class Geometry:
    """Acquisition geometry (Section 4.2): blade angles and widths, blade times, spectral axis."""
    n: int
    n_spec: int
    n_time: int
    angle_rad: np.ndarray
    lines: np.ndarray
    blade_time: Optional[np.ndarray]
    spec_shift_px: np.ndarray

    @classmethod
    def from_dict(cls, g: dict) -> "Geometry":
        bt = g.get("blade_time")
        return cls(n=int(g["n"]), n_spec=int(g["n_spec"]), n_time=int(g["n_time"]),
                   angle_rad=np.asarray(g["angle_rad"], dtype=np.float64),
                   lines=np.asarray(g["lines"], dtype=np.int64),
                   blade_time=None if bt is None else np.asarray(bt, dtype=np.float64),
                   spec_shift_px=np.asarray(g["spec_shift_px"], dtype=np.float64))

    @property
    def n_blades(self) -> int:
        return int(self.angle_rad.shape[0])

    def tau(self, b: int) -> float:
        return 0.0 if self.blade_time is None else float(self.blade_time[b])


def signed_freq(n: int) -> np.ndarray:
    """Signed DFT frequency of each unshifted index (reading R5)."""
    j = np.arange(n)
    return np.where(j <= (n - 1) // 2, j, j - n).astype(np.float64)


def blade_mask(n: int, theta: float, lines: int) -> np.ndarray:
    """k-space support of one blade (Section 4.2 "Blur"; Cartesian masks, Section 7; reading R6).

    A sample (ky, kx) is on the blade when its coordinate along the readout
    r = kx cos(theta) + ky sin(theta) lies in [-n/2, n/2) and its coordinate
    across the lines q = -kx sin(theta) + ky cos(theta) lies in [-L/2, L/2),
    both shifted by -1e-9 so that exact ties fall on one side.
    """
    k = signed_freq(n)
    ky, kx = np.meshgrid(k, k, indexing="ij")
    c, s = math.cos(theta), math.sin(theta)
    r = kx * c + ky * s
    q = -kx * s + ky * c
    e = MASK_EPS
    return (r >= -n / 2.0 - e) & (r < n / 2.0 - e) & (q >= -lines / 2.0 - e) & (q < lines / 2.0 - e)


def blade_masks(geom: Geometry) -> np.ndarray:
    return np.stack([blade_mask(geom.n, float(geom.angle_rad[b]), int(geom.lines[b]))
                     for b in range(geom.n_blades)])


def displacement(theta: float, delta: float) -> tuple[float, float]:
    """In-plane displacement (dx, dy) of spectral height delta seen by a blade at angle theta.

    Section 3: a constant frequency offset translates the image along the blade's
    readout direction; Section 4.2: the shift grows with spectral height (R1, R2).
    """
    return delta * math.cos(theta), delta * math.sin(theta)


# --------------------------------------------------------------------------- projection

def taps(d: tuple[float, float]) -> list[tuple[int, int, float]]:
    """Bilinear taps of a sample at (x - dx, y - dy): (row offset, column offset, weight).

    Section 4.2 "Projection": each ray sample is evaluated by interpolation into
    the volume (reading R3: bilinear in-plane at integer spectral planes).
    """
    dx, dy = d
    ox = math.floor(-dx)
    fx = -dx - ox
    oy = math.floor(-dy)
    fy = -dy - oy
    return [(oy, ox, (1.0 - fy) * (1.0 - fx)),
            (oy, ox + 1, (1.0 - fy) * fx),
            (oy + 1, ox, fy * (1.0 - fx)),
            (oy + 1, ox + 1, fy * fx)]


def _span(n: int, off: int) -> tuple[int, int]:
    """Output indices i in [lo, hi) whose tap i + off lies inside [0, n)."""
    return max(0, -off), min(n, n - off)


def shear(x: np.ndarray, d: tuple[float, float]) -> np.ndarray:
    """Sh(X; d): X resampled so that material at r appears at r + d; zero outside (R4)."""
    n = x.shape[-1]
    out = np.zeros_like(x, dtype=np.complex128)
    for ty, tx, w in taps(d):
        y0, y1 = _span(n, ty)
        x0, x1 = _span(n, tx)
        if y0 < y1 and x0 < x1:
            out[..., y0:y1, x0:x1] += w * x[..., y0 + ty:y1 + ty, x0 + tx:x1 + tx]
    return out


def shear_transpose(g: np.ndarray, d: tuple[float, float]) -> np.ndarray:
    """Sh^T(G; d): the transpose of ``shear``'s tap matrix, written as a literal scatter."""
    n = g.shape[-1]
    out = np.zeros_like(g, dtype=np.complex128)
    for ty, tx, w in taps(d):
        y0, y1 = _span(n, ty)
        x0, x1 = _span(n, tx)
        if y0 < y1 and x0 < x1:
            out[..., y0 + ty:y1 + ty, x0 + tx:x1 + tx] += w * g[..., y0:y1, x0:x1]
    return out


def knot_weights(tau: float, n_time: int) -> tuple[int, float]:
    """Time knot k and blend weight a of a blade at time tau (reading R11)."""
    if n_time == 1:
        return 0, 0.0
    u = tau * (n_time - 1)
    k = min(int(math.floor(u)), n_time - 2)
    return k, u - k


def volume_at(vol: np.ndarray, tau: float) -> np.ndarray:
    """The [S][n][n] volume a blade at time tau sees: linear blend of two knots (R11)."""
    t = vol.shape[0]
    k, a = knot_weights(tau, t)
    if t == 1:
        return vol[0].astype(np.complex128)
    return (1.0 - a) * vol[k] + a * vol[k + 1]


def project_blade(vol_s: np.ndarray, geom: Geometry, b: int) -> np.ndarray:
    """P_b = sum over spectral bins of the bin's image shifted by delta_s u_b (Section 4.2)."""
    theta = float(geom.angle_rad[b])
    out = np.zeros(vol_s.shape[-2:], dtype=np.complex128)
    for s in range(geom.n_spec):
        out += shear(vol_s[s], displacement(theta, float(geom.spec_shift_px[s])))
    return out


def forward_blade(vol: np.ndarray, geom: Geometry, b: int, mask: Optional[np.ndarray] = None) -> np.ndarray:
    """M_b . DFT2(P_b) with a unitary DFT (Section 4.2 "Blur", R5)."""
    if mask is None:
        mask = blade_mask(geom.n, float(geom.angle_rad[b]), int(geom.lines[b]))
    p = project_blade(volume_at(vol, geom.tau(b)), geom, b)
    return mask * np.fft.fft2(p, norm="ortho")


def forward(vol: np.ndarray, geom: Geometry, blades: Optional[Sequence[int]] = None) -> np.ndarray:
    """The measurement operator A: [T][S][n][n] -> [B][n][n] masked k-space (zeros for skipped blades)."""
    masks = blade_masks(geom)
    out = np.zeros((geom.n_blades, geom.n, geom.n), dtype=np.complex128)
    for b in (range(geom.n_blades) if blades is None else blades):
        out[b] = forward_blade(vol, geom, b, masks[b])
    return out


def residual(vol: np.ndarray, geom: Geometry, y: np.ndarray, blades: Optional[Sequence[int]] = None) -> np.ndarray:
    """R_b = M_b . K_b - M_b . y_b for the chosen blades; zero for the others (Section 4.3)."""
    masks = blade_masks(geom)
    out = np.zeros((geom.n_blades, geom.n, geom.n), dtype=np.complex128)
    for b in (range(geom.n_blades) if blades is None else blades):
        out[b] = forward_blade(vol, geom, b, masks[b]) - masks[b] * y[b].astype(np.complex128)
    return out


def data_loss(res: np.ndarray) -> float:
    """Half the squared L2 norm of the k-space residual (Section 4.3, reading R7)."""
    return 0.5 * float(np.sum(np.abs(res) ** 2))


def adjoint(kres: np.ndarray, geom: Geometry, blades: Optional[Sequence[int]] = None) -> np.ndarray:
    """A^H applied to a [B][n][n] k-space array: mask, unitary inverse DFT, transposed shear.

    For a real loss L(V) = 0.5 ||A V - y||^2 this returns dL/dRe V + i dL/dIm V.
    The shear transpose is the literal scatter of ``shear_transpose``; a dynamic
    blade's contribution is split onto its two knots with weights (1-a, a).
    """
    masks = blade_masks(geom)
    grad = np.zeros((geom.n_time, geom.n_spec, geom.n, geom.n), dtype=np.complex128)
    for b in (range(geom.n_blades) if blades is None else blades):
        g = np.fft.ifft2(masks[b] * kres[b].astype(np.complex128), norm="ortho")
        theta = float(geom.angle_rad[b])
        per_bin = np.stack([shear_transpose(g, displacement(theta, float(geom.spec_shift_px[s])))
                            for s in range(geom.n_spec)])
        if geom.n_time == 1:
            grad[0] += per_bin
        else:
            k, a = knot_weights(geom.tau(b), geom.n_time)
            grad[k] += (1.0 - a) * per_bin
            grad[k + 1] += a * per_bin
    return grad


# --------------------------------------------------------------------------- regularisers

def _charbonnier(z: np.ndarray, eps: float) -> np.ndarray:
    return np.sqrt(np.abs(z) ** 2 + eps * eps) - eps


def tv_value(vol: np.ndarray, eps: float) -> float:
    """Total variation over every axis of the volume (Section 4.3, reading R8)."""
    total = 0.0
    for axis in range(vol.ndim):
        if vol.shape[axis] > 1:
            total += float(np.sum(_charbonnier(np.diff(vol, axis=axis), eps)))
    return total


def tv_grad(vol: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of ``tv_value`` (dL/dRe + i dL/dIm)."""
    grad = np.zeros_like(vol, dtype=np.complex128)
    for axis in range(vol.ndim):
        if vol.shape[axis] < 2:
            continue
        d = np.diff(vol, axis=axis)
        w = d / np.sqrt(np.abs(d) ** 2 + eps * eps)
        hi = [slice(None)] * vol.ndim
        lo = [slice(None)] * vol.ndim
        hi[axis] = slice(1, None)
        lo[axis] = slice(None, -1)
        grad[tuple(hi)] += w
        grad[tuple(lo)] -= w
    return grad


def l1_value(vol: np.ndarray, eps: float) -> float:
    """L1 sparsity term (Section 4.3), Charbonnier-smoothed modulus (R8)."""
    return float(np.sum(_charbonnier(vol, eps)))


def l1_grad(vol: np.ndarray, eps: float) -> np.ndarray:
    return vol / np.sqrt(np.abs(vol) ** 2 + eps * eps)


def objective(vol: np.ndarray, geom: Geometry, y: np.ndarray, tv_weight: float, tv_eps: float,
              l1_weight: float = 0.0, blades: Optional[Sequence[int]] = None, data_weight: float = 1.0) -> float:
    """Weighted data term plus weighted TV and L1 (Section 4.3, R16)."""
    val = data_weight * data_loss(residual(vol, geom, y, blades))
    if tv_weight != 0.0:
        val += tv_weight * tv_value(vol, tv_eps)
    if l1_weight != 0.0:
        val += l1_weight * l1_value(vol, tv_eps)
    return val


def gradient(vol: np.ndarray, geom: Geometry, y: np.ndarray, tv_weight: float, tv_eps: float,
             l1_weight: float = 0.0, blades: Optional[Sequence[int]] = None,
             data_weight: float = 1.0) -> tuple[np.ndarray, float]:
    """Gradient of ``objective`` and the (weighted) data term at ``vol``."""
    res = residual(vol, geom, y, blades)
    g = data_weight * adjoint(res, geom, blades)
    if tv_weight != 0.0:
        g += tv_weight * tv_grad(vol, tv_eps)
    if l1_weight != 0.0:
        g += l1_weight * l1_grad(vol, tv_eps)
    return g, data_weight * data_loss(res)


# --------------------------------------------------------------------------- optimiser

def adam_update(vol: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
                lr: float, beta1: float, beta2: float, eps: float):
    """One Adam step (Kingma and Ba, Algorithm 1) on (Re, Im) as real parameters (R9).

    ``m`` and ``v`` have shape vol.shape + (2,): the first and second moments of
    the real and imaginary parts.
    """
    g = np.stack([grad.real, grad.imag], axis=-1)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    step = lr * mhat / (np.sqrt(vhat) + eps)
    return vol - (step[..., 0] + 1j * step[..., 1]), m, v


def gd_update(vol: np.ndarray, grad: np.ndarray, lr: float) -> np.ndarray:
    return vol - lr * grad


_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the output for state x, i.e. the
    mix of x + 0x9E3779B97F4A7C15."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def random_blade(seed: int, step_index: int, n_blades: int) -> int:
    """Blade of the random one-blade schedule at 0-based step index (R10)."""
    return splitmix64(((seed & 0xFFFFFFFF) << 32) | (step_index & 0xFFFFFFFF)) % n_blades


def reconstruct(geom: Geometry, y: np.ndarray, n_steps: int, tv_weight: float = 1e-3,
                tv_eps: float = 1e-3, l1_weight: float = 0.0, lr: float = 1e-2,
                beta1: float = 0.9, beta2: float = 0.999, adam_eps: float = 1e-8,
                optimizer: str = "adam", schedule: str = "all", init: Optional[np.ndarray] = None,
                split_bin: int = -1, state: Optional[dict] = None, seed: int = 0,
                data_weight: float = 1.0) -> dict:
    """The iterative fit of Section 4.3, from zero (or ``init``) for ``n_steps`` updates.

    ``state`` resumes a previous run: a dict with keys vol, m, v, step.
    Returns the volume, the renders, the pre-update objective of every step and
    the objective at the returned volume.
    """
    shape = (geom.n_time, geom.n_spec, geom.n, geom.n)
    if state is not None:
        vol = state["vol"].astype(np.complex128).copy()
        m = state["m"].copy()
        v = state["v"].copy()
        t0 = int(state["step"])
    else:
        vol = np.zeros(shape, dtype=np.complex128) if init is None else init.astype(np.complex128).copy()
        m = np.zeros(shape + (2,))
        v = np.zeros(shape + (2,))
        t0 = 0
    y = y.astype(np.complex128)
    history = []
    for t in range(t0 + 1, t0 + n_steps + 1):
        if schedule == "all":
            blades = None
        elif schedule == "cyclic":
            blades = [(t - 1) % geom.n_blades]
        else:
            blades = [random_blade(seed, t - 1, geom.n_blades)]
        g, ld = gradient(vol, geom, y, tv_weight, tv_eps, l1_weight, blades, data_weight)
        obj = ld
        if tv_weight != 0.0:
            obj += tv_weight * tv_value(vol, tv_eps)
        if l1_weight != 0.0:
            obj += l1_weight * l1_value(vol, tv_eps)
        history.append(obj)
        if optimizer == "adam":
            vol, m, v = adam_update(vol, g, m, v, t, lr, beta1, beta2, adam_eps)
        else:
            vol = gd_update(vol, g, lr)
    proj, water, fat = render(vol, split_bin)
    return dict(vol=vol, m=m, v=v, step=t0 + n_steps, proj=proj, water=water, fat=fat,
                history=np.asarray(history),
                final_loss=objective(vol, geom, y, tv_weight, tv_eps, l1_weight, data_weight=data_weight))


# --------------------------------------------------------------------------- outputs

def render(vol: np.ndarray, split_bin: int = -1):
    """Render with phi = 0 (Section 4.3) and split the spectral axis (Section 6, R12).

    proj[t] = sum over all bins; water = bins below the split; fat = the rest.
    """
    s = vol.shape[1]
    split = s // 2 if split_bin < 0 else split_bin
    proj = vol.sum(axis=1)
    water = vol[:, :split].sum(axis=1)
    fat = vol[:, split:].sum(axis=1)
    return proj, water, fat


def coverage_baseline(y: np.ndarray, masks: np.ndarray) -> np.ndarray:
    """Section 6: coverage-weighted average of the blades in k-space, then unitary inverse DFT."""
    cover = masks.sum(axis=0).astype(np.float64)
    acc = (masks * y.astype(np.complex128)).sum(axis=0)
    return np.fft.ifft2(acc / np.maximum(1.0, cover), norm="ortho")


def window_baseline(y: np.ndarray, masks: np.ndarray, window: int) -> np.ndarray:
    """Section 6, dynamic baseline: frame i is the coverage-weighted average, in k-space,
    of the blades i - window + 1 .. i (those that exist), then the unitary inverse DFT.
    Frames [B][n][n]; with window >= B the last frame is the static baseline."""
    B = y.shape[0]
    frames = np.zeros(y.shape, dtype=np.complex128)
    for i in range(B):
        lo = max(0, i - window + 1)
        frames[i] = coverage_baseline(y[lo:i + 1], masks[lo:i + 1])
    return frames


def psnr(image: np.ndarray, truth: np.ndarray) -> float:
    """PSNR on magnitudes with the peak of the truth (quality context only)."""
    err = np.mean((np.abs(image) - np.abs(truth)) ** 2)
    peak = float(np.max(np.abs(truth)))
    return float("inf") if err == 0 else 10.0 * math.log10(peak * peak / err)


# --------------------------------------------------------------------------- data

def simulate_measurements(case, dtype=np.complex64) -> np.ndarray:
    """Section 5: measure the ground-truth volume with the forward model, add noise.

    For every blade b at time tau_b: y_b = M_b . (DFT2(P_b V_GT(tau_b)) + sigma n_b),
    with V_GT(tau) the phantom's water layer on bin S/4 and fat on bin 3S/4
    rendered at that time. Returned in ``dtype`` (complex64, as the HIP path reads it).
    """
    from synth.phantom import ground_truth_volume

    geom = Geometry.from_dict(case.geometry())
    masks = blade_masks(geom)
    y = np.zeros((geom.n_blades, geom.n, geom.n), dtype=np.complex128)
    static_vol = None
    for b in range(geom.n_blades):
        tau = geom.tau(b)
        if geom.n_time == 1 and static_vol is not None:
            gt = static_vol
        else:
            w, f = case.layers_at(tau)
            gt = ground_truth_volume(w, f, geom.n_spec)
            if geom.n_time == 1:
                static_vol = gt
        p = project_blade(gt, geom, b)
        y[b] = masks[b] * (np.fft.fft2(p, norm="ortho") + case.sigma * case.noise[b])
    return y.astype(dtype)
