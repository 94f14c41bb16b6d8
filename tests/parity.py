"""Comparison helpers of the parity tests (HIP path against the FP64 oracle).

Two bounds hold together for every compared array:
  * relative L2 over the whole array, ||got - want|| / ||want||;
  * a per-element bound, max |got - want| <= tol * max |want|, which an error confined
    to a border row, one blade or one bin cannot hide from (in an array of 10^6 values
    such an error barely moves the whole-array norm).
"""

from __future__ import annotations

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
