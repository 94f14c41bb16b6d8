"""Sweep the fit's learning rate and TV weight on the FP64 oracle and record image quality.

For a static workload (the 64^2 or 256^2 one) this runs the oracle's Adam fit of
Section 4.3 from zero for the workload's step count at every (lr, TV weight) of a grid
and reports the PSNR on magnitudes of the render against the phantom's W + F, beside
the PSNR of the coverage-weighted baseline of Section 6 (quality context, not parity).
Only ``oracle/`` and ``synth/`` are imported; the grid points run in parallel processes.

    python tests/golden/quality_sweep.py static_64  [--jobs 4]
    -> tests/golden/quality_sweep_static_64.json
"""

from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import configs  # noqa: E402

GRIDS = {
    "static_64": dict(lr=(3e-3, 1e-2, 3e-2, 1e-1), tv=(1e-3, 3e-3, 1e-2, 3e-2, 1e-1)),
    "static_256": dict(lr=(1e-2, 3e-2), tv=(1e-3, 1e-2, 3e-2)),
}


def _keep_freed_memory() -> None:
    # large temporaries are served from a heap that keeps freed memory (no fresh page
    # faults for every one); where memory comes from, not any value, changes
    import ctypes

    libc = ctypes.CDLL("libc.so.6")
    libc.mallopt(-4, 0)
    libc.mallopt(-1, 2 ** 31 - 1)


def _truth(case):
    w, f = case.layers_at(0.0)
    return (w + f).astype(np.complex128)


def _point(args):
    name, lr, tv = args
    case = configs.CONFIGS[name]()
    geom = O.Geometry.from_dict(case.geometry())
    y = O.simulate_measurements(case)
    t0 = time.perf_counter()
    out = O.reconstruct(geom, y, case.n_steps, tv_weight=tv, tv_eps=case.tv_eps, lr=lr)
    p = O.psnr(out["proj"][0], _truth(case))
    print(f"[{name}] lr {lr:g} tv {tv:g}: psnr {p:.3f} dB ({time.perf_counter() - t0:.0f} s)", flush=True)
    return dict(lr=lr, tv_weight=tv, psnr_db=p, objective=float(out["final_loss"]))


def main() -> None:
    _keep_freed_memory()
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(GRIDS))
    ap.add_argument("--jobs", type=int, default=4)
    args = ap.parse_args()
    name = args.workload
    case = configs.CONFIGS[name]()
    y = O.simulate_measurements(case)
    base = O.psnr(O.coverage_baseline(y, O.blade_masks(O.Geometry.from_dict(case.geometry()))), _truth(case))
    grid = GRIDS[name]
    pts = [(name, lr, tv) for lr, tv in itertools.product(grid["lr"], grid["tv"])]
    import multiprocessing as mp

    with mp.get_context("fork").Pool(args.jobs) as pool:
        res = pool.map(_point, pts)
    best = max(res, key=lambda r: r["psnr_db"])
    out = dict(workload=name, steps=case.n_steps, optimizer="adam", tv_eps=case.tv_eps,
               baseline_psnr_db=base, best=best, points=res,
               note="PSNR on magnitudes of the render against W + F (peak max|truth|); baseline: "
                    "coverage-weighted average of all blades, unitary inverse DFT")
    with open(os.path.join(HERE, f"quality_sweep_{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"[{name}] baseline {base:.3f} dB; best lr {best['lr']:g} tv {best['tv_weight']:g}: "
          f"{best['psnr_db']:.3f} dB", flush=True)


if __name__ == "__main__":
    main()
