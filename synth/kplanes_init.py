"""Seeded initial parameters for K-Planes fits.

The K-Planes recipe: the grids that span only space and the spectral axis start
uniform in [0.1, 0.5) (real), the three grids with a time axis start at 1 (so that a
static scene needs no time variation), and the decoder weights start at 0, so that
the decoded volume starts at zero like the voxel grid. Grids are listed scale by
scale in the order xy, x-omega, y-omega, xt, yt, omega-t, then the weights; this
module knows only their sizes.
"""

from __future__ import annotations

import numpy as np


def grid_sizes(n_spec: int, features: int, time_res: int, spatial_res) -> list:
    """(name, element count) of every grid in parameter order, then ("a", F)."""
    out = []
    for r in spatial_res:
        out += [("xy", r * r * features), ("xs", n_spec * r * features), ("ys", n_spec * r * features),
                ("xt", time_res * r * features), ("yt", time_res * r * features),
                ("st", time_res * n_spec * features)]
    out.append(("a", features))
    return out


def init_params(n_spec: int, features: int, time_res: int, spatial_res, seed: int = 0,
                decoder_scale: float = 0.0) -> np.ndarray:
    """Flat complex128 initial parameters (draws: one uniform block per static grid, in
    order; then, if decoder_scale > 0, complex normal decoder weights times it)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, size in grid_sizes(n_spec, features, time_res, spatial_res):
        if name in ("xy", "xs", "ys"):
            parts.append(rng.uniform(0.1, 0.5, size).astype(np.complex128))
        elif name == "a":
            a = np.zeros(size, dtype=np.complex128)
            if decoder_scale > 0.0:
                a = decoder_scale * (rng.standard_normal(size) + 1j * rng.standard_normal(size))
            parts.append(a)
        else:
            parts.append(np.ones(size, dtype=np.complex128))
    return np.concatenate(parts)
