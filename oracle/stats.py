"""Error measures for sampled estimates (oracle; test infrastructure only).

Section 5 claims the sampling estimator is unbiased; Section 6.2 measures
accuracy on motif profiles.  The count-level measures here compare estimates
with exact counts directly.
"""
from __future__ import annotations

import numpy as np


def mass_weighted_relative_error(est: np.ndarray, exact: np.ndarray) -> float:
    """sum_m |est_m - exact_m| / sum_m exact_m for one run."""
    exact = np.asarray(exact, dtype=np.float64)
    return float(np.abs(np.asarray(est, dtype=np.float64) - exact).sum() / exact.sum())


def mean_relative_error(runs: np.ndarray, exact: np.ndarray) -> float:
    """Mean over runs (rows) of the mass-weighted relative error."""
    return float(np.mean([mass_weighted_relative_error(r, exact) for r in runs]))


def per_class_relative_error(runs: np.ndarray, exact: np.ndarray, min_count: float = 1.0) -> float:
    """Mean over runs and over classes with exact count >= min_count of |est-exact|/exact."""
    exact = np.asarray(exact, dtype=np.float64)
    sel = exact >= min_count
    rel = np.abs(np.asarray(runs, dtype=np.float64)[:, sel] - exact[sel]) / exact[sel]
    return float(rel.mean())


def bias_z(runs: np.ndarray, exact: np.ndarray) -> np.ndarray:
    """Per class: (mean over runs - exact) / standard error of the mean (0 where sd is 0)."""
    runs = np.asarray(runs, dtype=np.float64)
    n = runs.shape[0]
    mean = runs.mean(axis=0)
    sd = runs.std(axis=0, ddof=1)
    out = np.zeros(runs.shape[1])
    nz = sd > 0
    out[nz] = (mean[nz] - np.asarray(exact, dtype=np.float64)[nz]) / (sd[nz] / np.sqrt(n))
    return out
