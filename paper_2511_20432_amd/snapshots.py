"""Temperature snapshots on horizontal planes through the part (the top
surface and planes below it), as the paper shows its fields.

Marshalling and bookkeeping only: every temperature is evaluated by the
library (sa_iga_eval_temperature_at: the inverse of the geometry map, then
T = T~ + T^ of Eq. 21 in its kernels); points outside the part come back
as NaN.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np


def plane(model, z: float, lo: Sequence[float], hi: Sequence[float], n: Tuple[int, int] = (128, 128),
          path: int = 0):
    """T on an n[0] x n[1] grid of the plane z over [lo, hi] (x, y): returns
    (x [n0], y [n1], T [n1, n0]) with NaN outside the part."""
    xs = np.linspace(lo[0], hi[0], n[0])
    ys = np.linspace(lo[1], hi[1], n[1])
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)
    T, _, _ = model.eval_temperature_at(pts, path)
    return xs, ys, T.reshape(X.shape)


def summary(xs, ys, T, threshold: float) -> dict:
    """Largest temperature, the grid points inside the part, and the area of
    the plane above `threshold` (grid cells counted)."""
    inside = ~np.isnan(T)
    cell = (xs[1] - xs[0]) * (ys[1] - ys[0]) if len(xs) > 1 and len(ys) > 1 else 0.0
    hot = inside & (np.nan_to_num(T, nan=-np.inf) > threshold)
    return {"max_K": float(np.nanmax(T)) if inside.any() else None, "points_inside": int(inside.sum()),
            "area_above_m2": float(hot.sum() * cell), "threshold_K": float(threshold)}
