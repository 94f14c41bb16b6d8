"""Named synthetic workloads: acquisition geometry, phantom recipe and fit settings.

Every workload is built from a seed by the generators in ``phantom.py``. The
spectral axis places water on bin S/4 (zero shift) and fat on bin 3S/4 (a shift of
``f`` pixels along the blade's readout direction):

    delta_s = (s - S/4) * 2 f / S    pixels per bin,  f = max(2, n/64).

This is the caller-supplied off-resonance axis of the method: the paper tilts
the projection by a small angle phi off the spectral axis (Section 4.2,
"Projection"), and delta_s = tan(phi) * omega_s; f/S*2 = 0.25 px per bin at
n=64..256 is an effective tilt of about 14 degrees.

Ellipse count n_ell = round(8 + (n - 64)/12) (8 at n=64, 24 at n=256).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .phantom import EllipsePhantom, draw_noise, draw_phantom

GOLDEN_ANGLE_DEG = 180.0 / ((1.0 + math.sqrt(5.0)) / 2.0)


def fat_shift(n: int) -> float:
    return float(max(2.0, n / 64.0))


def n_ellipses(n: int) -> int:
    return int(round(8 + (n - 64) / 12.0))


def spectral_axis(n_spec: int, f: float) -> np.ndarray:
    """Shift in pixels of each spectral bin: zero at bin S/4, f at bin 3S/4."""
    s = np.arange(n_spec, dtype=np.float64)
    return (s - n_spec / 4.0) * 2.0 * f / n_spec


@dataclasses.dataclass
class Case:
    """One reconstruction problem: geometry, phantom, noise and fit settings."""
    name: str
    seed: int
    n: int
    n_spec: int
    n_time: int
    angle_rad: np.ndarray
    lines: np.ndarray
    blade_time: Optional[np.ndarray]
    spec_shift_px: np.ndarray
    phantom: EllipsePhantom
    noise: np.ndarray           # complex128 [B][n][n], unit variance per component
    sigma: float
    n_steps: int
    tv_weight: float = 1e-3
    l1_weight: float = 0.0
    tv_eps: float = 1e-3
    lr: float = 1e-2

    @property
    def n_blades(self) -> int:
        return int(self.angle_rad.shape[0])

    def geometry(self) -> dict:
        return dict(n=self.n, n_spec=self.n_spec, n_time=self.n_time,
                    angle_rad=self.angle_rad.copy(), lines=self.lines.copy(),
                    blade_time=None if self.blade_time is None else self.blade_time.copy(),
                    spec_shift_px=self.spec_shift_px.copy())

    def blade_times_or_zero(self) -> np.ndarray:
        if self.blade_time is None:
            return np.zeros(self.n_blades)
        return self.blade_time

    def layers_at(self, tau: float):
        return self.phantom.layers(tau)


def _build(name: str, seed: int, rng: np.random.Generator, n: int, n_spec: int, n_time: int,
           angles_deg: np.ndarray, lines: np.ndarray, blade_time, sigma: float, n_steps: int,
           motion_amp: float = 0.0, f: Optional[float] = None, n_ell: Optional[int] = None) -> Case:
    f = fat_shift(n) if f is None else f
    n_ell = n_ellipses(n) if n_ell is None else n_ell
    shifts = spectral_axis(n_spec, f)
    dynamic = n_time > 1
    ph = draw_phantom(rng, n, n_ell, 0.3, float(np.max(np.abs(shifts))),
                      motion_amp=motion_amp, dynamic=dynamic)
    noise = draw_noise(rng, len(angles_deg), n)
    return Case(name=name, seed=seed, n=n, n_spec=n_spec, n_time=n_time,
                angle_rad=np.deg2rad(np.asarray(angles_deg, dtype=np.float64)),
                lines=np.asarray(lines, dtype=np.int32),
                blade_time=None if blade_time is None else np.asarray(blade_time, dtype=np.float64),
                spec_shift_px=shifts, phantom=ph, noise=noise, sigma=sigma, n_steps=n_steps)


def static_64(seed: int = 1001) -> Case:
    """64x64, S=16, five 16x64 blades at k*36 degrees, 200 steps."""
    rng = np.random.default_rng(seed)
    return _build("static_64", seed, rng, 64, 16, 1, 36.0 * np.arange(5), np.full(5, 16), None,
                  1e-3, 200)


def static_256(seed: int = 2001) -> Case:
    """256x256, S=32, twelve 32x256 blades uniform over 180 degrees, 500 steps."""
    rng = np.random.default_rng(seed)
    return _build("static_256", seed, rng, 256, 32, 1, 15.0 * np.arange(12), np.full(12, 32), None,
                  1e-3, 500)


def dynamic_192(seed: int = 3001) -> Case:
    """192x192, S=32, T=16 knots, 32 sequential golden-angle 24x192 blades, 800 steps."""
    rng = np.random.default_rng(seed)
    b = np.arange(32)
    angles = np.mod(b * GOLDEN_ANGLE_DEG, 180.0)
    return _build("dynamic_192", seed, rng, 192, 32, 16, angles, np.full(32, 24), b / 32.0,
                  2e-3, 800, motion_amp=6.0)


def batch_slice(j: int) -> Case:
    """Slice j of the 64-slice batch: size, depth, blade count and width drawn per seed."""
    seed = 4000 + j
    rng = np.random.default_rng(seed)
    n = int(rng.choice([128, 192, 256]))
    s = int(rng.choice([16, 32]))
    nb = int(rng.integers(8, 17))
    lines = int(rng.integers(16, 33))
    return _build(f"batch_{j}", seed, rng, n, s, 1, 180.0 * np.arange(nb) / nb, np.full(nb, lines),
                  None, 1e-3, 200)


def serving_request(i: int, base_seed: int = 5000) -> Case:
    """Request i of the served stream: static or dynamic, mixed sizes."""
    seed = base_seed + i
    rng = np.random.default_rng(seed)
    n = int(rng.choice([128, 192, 256, 320, 384]))
    s = int(rng.choice([16, 32, 64]))
    nb = int(rng.integers(8, 33))
    lines = int(rng.choice([16, 24, 32]))
    t = int(rng.choice([1, 8, 16]))
    if t == 1:
        angles = 180.0 * np.arange(nb) / nb
        return _build(f"serve_{i}", seed, rng, n, s, 1, angles, np.full(nb, lines), None, 1e-3, 200)
    b = np.arange(nb)
    angles = np.mod(b * GOLDEN_ANGLE_DEG, 180.0)
    return _build(f"serve_{i}", seed, rng, n, s, t, angles, np.full(nb, lines), b / nb, 2e-3, 800,
                  motion_amp=6.0)


def small_case(n: int = 48, n_spec: int = 6, n_time: int = 1, n_blades: int = 4, lines: int = 12,
               seed: int = 7, sigma: float = 1e-3, n_steps: int = 20, f: float = 2.0,
               motion_amp: float = 3.0) -> Case:
    """A small case for parity tests: sizes chosen to span several tiles and a ragged tail."""
    rng = np.random.default_rng(seed)
    if n_time > 1:
        b = np.arange(n_blades)
        angles = np.mod(b * GOLDEN_ANGLE_DEG, 180.0)
        times = b / float(n_blades)
    else:
        angles = 180.0 * np.arange(n_blades) / n_blades
        times = None
    return _build(f"small_{n}_{n_spec}_{n_time}", seed, rng, n, n_spec, n_time, angles,
                  np.full(n_blades, lines), times, sigma, n_steps,
                  motion_amp=motion_amp if n_time > 1 else 0.0, f=f,
                  n_ell=max(3, n_ellipses(n)))


CONFIGS = {
    "static_64": static_64,
    "static_256": static_256,
    "dynamic_192": dynamic_192,
}


def config_geometry(name: str) -> dict:
    return CONFIGS[name]().geometry()


def config_options(case: Case) -> dict:
    return dict(tv_weight=case.tv_weight, l1_weight=case.l1_weight, tv_eps=case.tv_eps,
                n_steps=case.n_steps, lr=case.lr, beta1=0.9, beta2=0.999, adam_eps=1e-8)
