"""Seeded synthetic inputs for lifted PROPELLER reconstruction.

This package draws the inputs that both the FP64 oracle and the HIP path consume:
acquisition geometry (blade angles, line counts, blade times, spectral shift axis),
ground-truth fat/water layers from a random-ellipse phantom, and the complex
Gaussian noise array. It holds none of the reconstruction arithmetic: no masks,
no projection, no DFT, no loss. The measurement itself is produced by whichever
side consumes these arrays, with its own forward model.
"""

from .configs import CONFIGS, config_geometry, config_options, spectral_axis, fat_shift, n_ellipses
from .phantom import EllipsePhantom, draw_phantom, draw_noise, ground_truth_volume

__all__ = [
    "CONFIGS",
    "config_geometry",
    "config_options",
    "spectral_axis",
    "fat_shift",
    "n_ellipses",
    "EllipsePhantom",
    "draw_phantom",
    "draw_noise",
    "ground_truth_volume",
]
