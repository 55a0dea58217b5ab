"""Evaluation at physical points (Eq. 21 after the inverse of the geometry
map) through the C ABI against the FP64 oracle: on the quarter annulus and on
the Table 2 part, T and grad T at 1e-9 (normwise) and the located parametric
points to 1e-10; points outside the patch give NaN on both sides."""
import math

import numpy as np
import pytest

from oracle import bspline, solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("which", ["annulus", "part"])
def test_physical_points_match_oracle(which):
    from paper_2511_20432_amd import sa_iga
    if which == "annulus":
        patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (12, 6, 4), 2)
        r = 3.88e-3
        a0, a1 = math.radians(20.0), math.radians(60.0)
        scan = W.single_track((r * math.cos(a0), r * math.sin(a0), 1e-3), (r * math.cos(a1), r * math.sin(a1), 1e-3),
                              80.0, 0.8, 1e-5, 8)
        mat, s, steps = W.MAT_CFG, 1.0, 25
    else:
        w = W.e2((3, 4, 6))
        patch, scan, mat, s, steps = w.patch, w.scan, w.material, 2.0, 150
    gm = sa_iga.Model(patch, mat, scan, W.Options(precision=W.PRECISION_FP64, kernel_scale=s))
    om = solver.Model(patch, mat, scan, kernel_scale=s)
    gm.step(steps)
    om.advance(steps)
    rng = np.random.default_rng(8)
    x_in = bspline.geometry(patch, rng.random((300, 3)))[0]
    lo, hi = x_in.min(axis=0), x_in.max(axis=0)
    x_out = np.array([hi + 1e-4, lo - 1e-4])
    x = np.concatenate([x_in, x_out])
    T, G, xi = gm.eval_temperature_at(x)
    Tr, Gr, xir = om.evaluate_at(x)
    assert np.isnan(T[-2:]).all() and np.isnan(xi[-2:]).all() and np.isnan(Tr[-2:]).all()
    k = slice(0, len(x_in))
    e = {"T": rel(T[k] - mat.T0, Tr[k] - mat.T0), "grad": rel(G[k], Gr[k]),
         "xi": float(np.abs(xi[k] - xir[k]).max())}
    print(f"{which}, step {steps}: {e}, max T {np.nanmax(T):.1f} K", flush=True)
    assert e["T"] <= 1e-9 and e["grad"] <= 1e-9 and e["xi"] <= 1e-10
