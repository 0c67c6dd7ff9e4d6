"""Helpers shared by the GPU tests: layout conversion and the exemption rule."""
from __future__ import annotations

import numpy as np

EXEMPT = 1e-5          # |dE - T| below which a device decision may differ from the FP64 oracle's


def natural(half) -> np.ndarray:
    """(2, L, L/2) half-lattice state (torch or numpy) -> (L, L) float64 array theta[y, x]."""
    if hasattr(half, "detach"):
        half = half.detach().float().cpu().numpy()
    half = np.asarray(half, dtype=np.float64)
    _, L, H = half.shape
    out = np.empty((L, L), dtype=np.float64)
    y = np.arange(L)[:, None]
    k = np.arange(H)[None, :]
    for c in (0, 1):
        x = 2 * k + ((c + y) & 1)
        out[np.broadcast_to(y, x.shape), x] = half[c]
    return out


def natural_u8(half) -> np.ndarray:
    if hasattr(half, "detach"):
        half = half.detach().cpu().numpy()
    return natural(half.astype(np.float64))


def exempt_mask(diag, L: int) -> np.ndarray:
    """Sites whose device decision may legitimately differ from the oracle's in one
    sweep: near-threshold sites, and black sites next to a near-threshold red site
    (their inputs may differ)."""
    near = np.abs(diag["dE"] - diag["thr"]) < EXEMPT
    y, x = np.mgrid[0:L, 0:L]
    red = ((x + y) & 1) == 0
    red_near = near & red
    spread = (red_near | np.roll(red_near, 1, 0) | np.roll(red_near, -1, 0) | np.roll(red_near, 1, 1)
              | np.roll(red_near, -1, 1))
    return near | (spread & ~red)


def obs_tol(ref: float, N: int) -> float:
    """Observable tolerance: 1e-6 relative, with N as the scale for sums near zero."""
    return 1e-6 * max(abs(ref), N)
