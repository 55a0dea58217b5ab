"""Full-size trajectories against the oracle's own: the raster block (cfg2,
cubic, 44,555 DOFs, every one of its 3,788 steps) and the quarter annulus
(cfg3, quadratic NURBS, 18,200 DOFs, its first 2,000 steps).  The oracle ran
each scan once from u = T_c on the CPU (tests/golden/make_trajectory_snapshots.py:
the FP64 kernel sum over every switched-on source at every lateral and
bottom point, the load vector of Eq. 18, the projection of Eq. 11 and the
theta-scheme of Eq. 20 with a sparse LU solve) and stored the control values
w = u - T_c and the load vector F at a few steps.

  * FP64 form: w and F at every stored step within 1e-9 (normwise);
  * FP32 far-field form: |T - T_oracle| <= |dT~| + max |dw| <= 0.05 K, with
    T~ at sampled boundary points from the oracle's kernel sum;
  * the heat-loss diagnostic (Sec. 3.1) along the top edge of the annulus's
    outer arc at a stored step, with the oracle's own control values.
"""
import os

import numpy as np
import pytest

from oracle import iga, pointsource, solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL64 = 1e-9
TOL_K = 0.05


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _snap(name):
    path = os.path.join(GOLDEN, f"traj_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_trajectory_snapshots.py {name})")
    with np.load(path, allow_pickle=False) as z:
        return z["steps"].copy(), z["w"].copy(), z["F"].copy()


def _workload(name):
    return W.cfg2(seed=0) if name == "cfg2" else W.cfg3(seed=0)


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_fp64_trajectory_matches_oracle(name):
    from paper_2511_20432_amd import sa_iga
    steps, w_ref, F_ref = _snap(name)
    w = _workload(name)
    gm = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP64))
    done = 0
    for k, s in enumerate(steps):
        gm.step(int(s) - done)
        done = int(s)
        _, _, F, du = gm.boundary_fields()
        e_w, e_F = rel(du, w_ref[k]), rel(F, F_ref[k])
        print(f"{name} FP64 step {s}: w rel {e_w:.2e} (max |w| {np.abs(w_ref[k]).max():.3e} K), F rel {e_F:.2e}",
              flush=True)
        assert e_w <= TOL64 and e_F <= TOL64


@pytest.mark.parametrize("name", ["cfg2", "cfg3"])
def test_fp32_far_trajectory_within_005K_of_oracle(name):
    from paper_2511_20432_amd import sa_iga
    steps, w_ref, _ = _snap(name)
    w = _workload(name)
    gm = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP32_FAR, tau_near=2e-4))
    bt = iga.boundary_tables(w.patch)
    rng = np.random.default_rng(5)
    q = np.sort(rng.choice(len(bt["x"]), 400, replace=False))
    sc = w.scan
    done = 0
    for k, s in enumerate(steps):
        gm.step(int(s) - done)
        done = int(s)
        T, _, _, du = gm.boundary_fields()
        Tr, _ = pointsource.field(bt["x"][q], sc.xyz, sc.tick, sc.energy, int(s), sc, w.material)
        e_T = float(np.abs(T[q] - Tr).max())
        e_w = float(np.abs(du - w_ref[k]).max())
        print(f"{name} FP32 far step {s}: max |dT~| {e_T:.2e} K (sampled), max |dw| {e_w:.2e} K", flush=True)
        assert e_T + e_w <= TOL_K


def test_heat_loss_at_full_size_matches_oracle():
    from paper_2511_20432_amd import sa_iga
    steps, w_ref, _ = _snap("cfg3")
    w = _workload("cfg3")
    s = int(steps[0])
    gm = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP64))
    gm.step(s)
    om = solver.Model(w.patch, w.material, w.scan, assemble=False)
    for face in (3, 1):
        g = gm.heat_loss(face, 5, quad=4)
        o = om.heat_loss(face, 5, quad=4, u=w.material.T0 + w_ref[0], step=s)
        errs = {k: rel(g[k], o[k]) for k in ("ds", "q_tilde", "q_hat")}
        errs["net"] = abs(g["net"] - o["net"]) / abs(o["net"])
        print(f"cfg3 step {s} face {face}: int|q~+q^| ds {g['net']:.4e} W/m, int|q~| ds {g['tilde']:.4e} W/m "
              f"(ratio {g['net'] / g['tilde']:.3f}); worst rel {max(errs.values()):.2e}", flush=True)
        assert max(errs.values()) <= TOL64
