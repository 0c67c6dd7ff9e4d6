"""Error bars for correlated Monte Carlo time series (binning analysis)."""
from __future__ import annotations

import numpy as np


def binned_error(x, min_bins: int = 32) -> float:
    """Standard error of the mean of a correlated series.

    Bins of size 1, 2, 4, ... are formed while at least ``min_bins`` bins remain;
    the error of the mean is estimated from the spread of the bin averages at each
    level, and the largest estimate over the levels is returned (the plateau value
    for a long enough series, a conservative bound otherwise).
    """
    x = np.asarray(x, dtype=np.float64)
    best = 0.0
    while x.size >= min_bins:
        err = x.std(ddof=1) / np.sqrt(x.size)
        best = max(best, err)
        n = x.size // 2
        x = 0.5 * (x[: 2 * n : 2] + x[1 : 2 * n : 2])
    return best


def mean_err(x, discard: int = 0):
    x = np.asarray(x, dtype=np.float64)[discard:]
    return float(x.mean()), binned_error(x)


def observables(rec: np.ndarray, N: int, beta: float):
    """Per-record series from raw records [sweep, acc, Cx, Cy, Ix, Iy, Mx, My]:
    energy per site, |m| per site, and the helicity-modulus estimator
    (Cx + Cy - beta (Ix^2 + Iy^2)) / (2N) whose mean is the helicity modulus."""
    cx, cy, ix, iy, mx, my = (rec[:, k] for k in range(2, 8))
    e = -(cx + cy) / N
    m = np.hypot(mx, my) / N
    ups = (cx + cy - beta * (ix * ix + iy * iy)) / (2.0 * N)
    return e, m, ups
