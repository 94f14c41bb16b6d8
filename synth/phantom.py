"""Random-ellipse fat/water phantom and measurement noise.

The paper builds its ground truth by embedding fat and water layers along the
spectral axis of a volume (Section 5, "Datasets"); its own Shepp-Logan layers and
the Dixon-RAVE data are not reproduced here. A seed-drawn set of random ellipses
stands in: every ellipse carries water, a fixed fraction also carries fat, and for
dynamic scans every ellipse translates sinusoidally along x (the "left and right"
motion of the dynamic Shepp-Logan dataset, Section 5).

Draw order (NumPy PCG64, FP64) is fixed so that every consumer sees the same case:
  1. per ellipse: semi-axes a, b ~ U(0.05 n, 0.20 n); rotation psi ~ U(0, pi);
     centre x then y ~ U(n/2 - R, n/2 + R) with R = n/2 - max(a, b) - margin;
     water amplitude ~ U(0.2, 1);
  2. fat set = permutation(n_ell)[:round(fat_fraction * n_ell)], fat amplitudes
     ~ U(0.2, 0.8) in that order;
  3. dynamic only: per-ellipse motion phase ~ U(0, 2 pi);
  4. the noise array, last (``draw_noise``).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class EllipsePhantom:
    n: int
    a: np.ndarray          # semi-axis along the rotated x' axis (pixels)
    b: np.ndarray          # semi-axis along the rotated y' axis (pixels)
    psi: np.ndarray        # rotation (radians)
    cx: np.ndarray         # centre column (pixels)
    cy: np.ndarray         # centre row (pixels)
    water: np.ndarray      # water amplitude per ellipse
    fat: np.ndarray        # fat amplitude per ellipse (0 where the ellipse has no fat)
    phase: np.ndarray      # motion phase per ellipse (zeros for static phantoms)
    motion_amp: float      # peak x displacement in pixels (0 for static phantoms)

    @property
    def n_ellipses(self) -> int:
        return int(self.a.shape[0])

    def centres_at(self, tau: float) -> tuple[np.ndarray, np.ndarray]:
        """Centres at scan time tau in [0, 1]: one period of sinusoidal x motion."""
        dx = self.motion_amp * np.sin(2.0 * math.pi * tau + self.phase)
        return self.cx + dx, self.cy

    def layers(self, tau: float = 0.0) -> tuple[np.ndarray, np.ndarray]:
        """Rasterise the (water, fat) layers at time tau as complex128 [n][n] images.

        A pixel centre (integer x = column, y = row) is inside an ellipse when its
        quadratic form is <= 1; amplitudes of overlapping ellipses add.
        """
        n = self.n
        yy, xx = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64), indexing="ij")
        cx, cy = self.centres_at(tau)
        water = np.zeros((n, n), dtype=np.complex128)
        fat = np.zeros((n, n), dtype=np.complex128)
        for e in range(self.n_ellipses):
            c, s = math.cos(self.psi[e]), math.sin(self.psi[e])
            u = (xx - cx[e]) * c + (yy - cy[e]) * s
            v = -(xx - cx[e]) * s + (yy - cy[e]) * c
            inside = (u / self.a[e]) ** 2 + (v / self.b[e]) ** 2 <= 1.0
            water[inside] += self.water[e]
            if self.fat[e] != 0.0:
                fat[inside] += self.fat[e]
        return water, fat


def draw_phantom(rng: np.random.Generator, n: int, n_ell: int, fat_fraction: float,
                 max_abs_shift: float, motion_amp: float = 0.0, dynamic: bool = False) -> EllipsePhantom:
    """Draw a random-ellipse phantom from ``rng`` in the documented order."""
    margin = math.ceil(max_abs_shift) + 2 + motion_amp
    a = np.empty(n_ell)
    b = np.empty(n_ell)
    psi = np.empty(n_ell)
    cx = np.empty(n_ell)
    cy = np.empty(n_ell)
    water = np.empty(n_ell)
    for e in range(n_ell):
        a[e] = rng.uniform(0.05 * n, 0.20 * n)
        b[e] = rng.uniform(0.05 * n, 0.20 * n)
        psi[e] = rng.uniform(0.0, math.pi)
        r = max(0.0, n / 2.0 - max(a[e], b[e]) - margin)
        cx[e] = rng.uniform(n / 2.0 - r, n / 2.0 + r)
        cy[e] = rng.uniform(n / 2.0 - r, n / 2.0 + r)
        water[e] = rng.uniform(0.2, 1.0)
    n_fat = int(round(fat_fraction * n_ell))
    fat_set = rng.permutation(n_ell)[:n_fat]
    fat = np.zeros(n_ell)
    for e in fat_set:
        fat[e] = rng.uniform(0.2, 0.8)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_ell) if dynamic else np.zeros(n_ell)
    return EllipsePhantom(n=n, a=a, b=b, psi=psi, cx=cx, cy=cy, water=water, fat=fat,
                          phase=phase, motion_amp=float(motion_amp if dynamic else 0.0))


def draw_noise(rng: np.random.Generator, n_blades: int, n: int) -> np.ndarray:
    """Unit complex Gaussian noise n1 + i n2 per k-space sample, complex128 [B][n][n]."""
    re = rng.standard_normal((n_blades, n, n))
    im = rng.standard_normal((n_blades, n, n))
    return re + 1j * im


def ground_truth_volume(water: np.ndarray, fat: np.ndarray, n_spec: int) -> np.ndarray:
    """Embed the layers along the spectral axis: water on bin S/4, fat on bin 3S/4.

    Returns complex128 [S][n][n]. With the spectral axis of ``configs.spectral_axis``
    bin S/4 has zero shift and bin 3S/4 the full fat shift.
    """
    n = water.shape[-1]
    vol = np.zeros((n_spec, n, n), dtype=np.complex128)
    vol[n_spec // 4] += water
    vol[(3 * n_spec) // 4] += fat
    return vol
