"""Write the converged-image fixtures of the full-size workloads from the FP64 oracle.

For the static 256^2 workload (S 32, 12 blades, 500 Adam steps), the dynamic 192^2
workload (S 32, T 16, 32 blades, 800 Adam steps), a slice of the 64-slice batch or a
request of the served stream (each with its own steps and settings) this runs the
oracle's fit of
Section 4.3 from zero on the seeded measurements and stores the rendered complex
image (Section 4.3, the render at phi = 0) and the final objective:

    tests/golden/converged_<workload>.npz   proj (complex64 [T][n][n]), final_loss,
                                            steps, and the image at a few earlier steps

Only ``oracle/`` and ``synth/`` are imported. The fit is run in chunks that resume from
the previous chunk's state (the resume is bitwise, so this is the same fit).

``--spread`` also runs the fit (in parallel processes) on the same measurements
perturbed at FP32 rounding level and 16 times that, y (1 + 2^-24 z) and y (1 + 2^-20 z)
with z complex standard normal, and reports, at each checkpoint, the relative L2
distance between the perturbed and the unperturbed render and the largest element
difference relative to the largest element: how far an FP32 evaluation of the fit,
whose operator and data carry rounding errors of that size, can be expected to wander
from the FP64 one. It writes ``converged_<workload>_spread.json`` beside the fixture.

Run from the repository root:  python tests/golden/make_converged.py static_256 [--spread]
"""

from __future__ import annotations

import argparse
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


def _keep_freed_memory() -> None:
    """Serve every allocation from the heap and never hand freed memory back.

    The fit allocates volume-sized temporaries (300 MB at 192^2 x 32 x 16) many times
    per step; glibc maps each one afresh by default, and first-touch page faults then
    cost more than the arithmetic. This changes where memory comes from, not any value.
    """
    import ctypes

    libc = ctypes.CDLL("libc.so.6")
    libc.mallopt(-4, 0)              # M_MMAP_MAX: no mmap'd chunks
    libc.mallopt(-1, 2 ** 31 - 1)    # M_TRIM_THRESHOLD: keep freed heap memory

CHECKPOINTS = (1, 3, 10, 30, 100, 300)


def rel(a, b) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_fit(case, y, label: str):
    """The oracle's Adam fit with the workload's settings; renders at the checkpoints."""
    geom = O.Geometry.from_dict(case.geometry())
    marks = [c for c in CHECKPOINTS if c < case.n_steps] + [case.n_steps]
    state = None
    done = 0
    images = {}
    objectives = {}
    t0 = time.perf_counter()
    for mark in marks:
        out = O.reconstruct(geom, y, mark - done, tv_weight=case.tv_weight, tv_eps=case.tv_eps,
                            l1_weight=case.l1_weight, lr=case.lr, state=state)
        state = dict(vol=out["vol"], m=out["m"], v=out["v"], step=out["step"])
        done = mark
        images[mark] = out["proj"]
        objectives[mark] = float(out["final_loss"])
        print(f"[{label}] step {mark}/{case.n_steps} objective {out['final_loss']:.9e} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    return images, objectives


PERTURB_LOG2 = (-24, -20)


def max_rel(a, b) -> float:
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def case_for(name: str):
    """A named workload, a slice of the 64-slice batch (batch_<j>) or a request of the
    served stream (serve_<i>)."""
    if name.startswith("batch_"):
        return configs.batch_slice(int(name[6:]))
    if name.startswith("serve_"):
        return configs.serving_request(int(name[6:]))
    return configs.CONFIGS[name]()


def _fit_worker(args):
    name, log2 = args
    case = case_for(name)
    y = O.simulate_measurements(case)
    label = name
    if log2 is not None:
        rng = np.random.default_rng(12345)
        z = rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)
        y = y.astype(np.complex128) * (1.0 + 2.0 ** log2 * z)
        label += f" perturbed 2^{log2}"
    return run_fit(case, y, label)


def main() -> None:
    _keep_freed_memory()
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", help="static_64, static_256, dynamic_192, batch_<j> or serve_<i>")
    ap.add_argument("--spread", action="store_true",
                    help="also fit the perturbed measurements (in a second process) and report the spread")
    args = ap.parse_args()
    name = args.workload
    case = case_for(name)
    jobs = [(name, None)] + ([(name, k) for k in PERTURB_LOG2] if args.spread else [])
    if len(jobs) == 1:
        results = [_fit_worker(jobs[0])]
    else:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(len(jobs)) as pool:
            results = pool.map(_fit_worker, jobs)
    images, objectives = results[0]
    final_loss = objectives[case.n_steps]
    extra = {f"proj_step{k}": v.astype(np.complex64) for k, v in images.items() if k in (10, 100)}
    np.savez_compressed(os.path.join(HERE, f"converged_{name}.npz"),
                        proj=images[case.n_steps].astype(np.complex64),
                        final_loss=np.float64(final_loss), steps=np.int64(case.n_steps), **extra)
    if args.spread:
        out = dict(workload=name, perturbation="y * (1 + 2^k z), z complex standard normal (seed 12345)",
                   checkpoints=sorted(images), objective={str(c): objectives[c] for c in images})
        for k, res in zip(PERTURB_LOG2, results[1:]):
            pert = res[0]
            out[f"rel_l2_2^{k}"] = {str(c): rel(pert[c], images[c]) for c in images}
            out[f"max_elem_2^{k}"] = {str(c): max_rel(pert[c], images[c]) for c in images}
            out[f"objective_rel_2^{k}"] = {str(c): abs(res[1][c] - objectives[c]) / abs(objectives[c]) for c in images}
            print(f"[{name}] 2^{k}: rel L2 {out[f'rel_l2_2^{k}']}; max elem {out[f'max_elem_2^{k}']}", flush=True)
        with open(os.path.join(HERE, f"converged_{name}_spread.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
