"""Comparison helpers of the parity tests (HIP path against the FP64 oracle).

Two bounds hold together for every compared array:
  * relative L2 over the whole array, ||got - want|| / ||want||;
  * a per-element bound, max |got - want| <= tol * max |want|, which an error confined
    to a border row, one blade or one bin cannot hide from (in an array of 10^6 values
    such an error barely moves the whole-array norm).
"""

from __future__ import annotations

import json
import os

import numpy as np


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_rel(a, b) -> float:
    """max |a - b| / max |b| (the per-element bound's ratio)."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    if b.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def both_bounds(a, b) -> float:
    """max(relative L2, per-element ratio): one number below a tolerance meets both bounds."""
    return max(rel(a, b), max_rel(a, b))


def assert_close(got, want, tol: float, what: str = "", elem_tol: float | None = None) -> tuple[float, float]:
    """Both bounds at `tol` (the per-element one at `elem_tol` if given); returns the two ratios."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    r, m = rel(got, want), max_rel(got, want)
    et = tol if elem_tol is None else elem_tol
    assert r < tol and m <= et, f"{what}: rel L2 {r:.3e} (tol {tol:.0e}), max elem {m:.3e} (tol {et:.0e})"
    return r, m


# Converged fits (Adam) against the oracle's stored renders (tests/golden/make_converged.py):
# the bound at a checkpoint is RECON_TOL or twice the oracle's own spread there, the
# distance its FP64 fit moves when y is perturbed at FP32 rounding level (y (1 + 2^-20 z)).
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RECON_TOL = 1e-3
SPREAD_LOG2 = -20
SPREAD_FACTOR = 2.0


def adam_tol(spread: float) -> float:
    return max(RECON_TOL, SPREAD_FACTOR * spread)


def stored_spread(name: str, step: int) -> tuple[float, float, float]:
    """The oracle's spread (rel L2 of proj, max element of proj, objective) at a
    checkpoint of a stored fit, from its 2^-20 perturbation run (skips the test if the
    fixture has not been generated)."""
    import pytest

    path = os.path.join(GOLDEN, f"converged_{name}_spread.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_converged.py {name} --spread)")
    with open(path) as fh:
        d = json.load(fh)
    k, c = SPREAD_LOG2, str(step)
    return (d[f"rel_l2_2^{k}"][c], d[f"max_elem_2^{k}"][c], d[f"objective_rel_2^{k}"][c])


def converged_fixture(name: str):
    """The oracle's stored renders of a fit (plain arrays; allow_pickle stays off)."""
    import pytest

    path = os.path.join(GOLDEN, f"converged_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_converged.py {name} --spread)")
    return np.load(path)


def check_converged(name: str, proj, objective, step=None):
    """A fit's render (and, at the last step, its objective) against the stored oracle fit
    at `step` (the last step when None); returns the ratios for printing."""
    ref = converged_fixture(name)
    last = int(ref["steps"])
    step = last if step is None else step
    want = (ref["proj"] if step == last else ref[f"proj_step{step}"]).astype(np.complex128)
    sr, se, so = stored_spread(name, step)
    r, m = assert_close(proj, want, adam_tol(sr), f"{name} proj at step {step}", elem_tol=adam_tol(se))
    out = dict(step=step, rel=r, max_elem=m, spread=sr, spread_elem=se)
    if objective is not None and step == last:
        want_obj = float(ref["final_loss"])
        rel_obj = abs(objective - want_obj) / abs(want_obj)
        assert rel_obj <= adam_tol(so), f"{name} objective {objective} vs {want_obj} (spread {so:.2e})"
        out.update(objective_rel=rel_obj, objective_spread=so)
    return out
