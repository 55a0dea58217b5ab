"""Parity at the benchmark's full size: the raster workload (44,555 DOFs,
64,512 boundary points) in the launch configuration bench.py times (one path,
tuned tile shape).  The oracle cannot run the whole scan, so it checks
sampled outputs one by one and the theta-scheme equation at sampled rows:

  * T~ and grad T~ at sampled boundary points (Eqs. 7-8),
  * the load vector at sampled lateral rows (Eqs. 10, 18),
  * the Dirichlet values: the oracle's own L2 projection (Eq. 11) of its own
    T~ at every bottom point,
  * (M/dt + theta K) w^{n+1} = (M/dt - (1-theta) K) w^n + theta F^{n+1}
    + (1-theta) F^n (Eq. 20) at sampled free rows, with rows of M and K the
    oracle assembles itself.
"""
import numpy as np
import pytest

from oracle import iga, pointsource, solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def raster_run():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg2(seed=0)
    gm = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP64))
    gm.autotune(reps=2)
    n = 301
    gm.step(n - 1)
    f0 = gm.boundary_fields()
    gm.step(1)
    f1 = gm.boundary_fields()
    om = solver.Model(w.patch, w.material, w.scan, assemble=False)
    return w, gm, om, n, f0, f1


def test_source_field_at_sampled_points(raster_run):
    w, gm, om, n, f0, f1 = raster_run
    T, G = f1[0], f1[1]
    rng = np.random.default_rng(11)
    q = np.sort(rng.choice(len(T), 600, replace=False))
    sc = w.scan
    Tr, Gr = pointsource.field(om.bt["x"][q], sc.xyz, sc.tick, sc.energy, n, sc, w.material)
    e_T, e_G = rel(T[q], Tr), rel(G[q], Gr)
    print(f"T~ rel {e_T:.2e}, grad rel {e_G:.2e} at {len(q)} points", flush=True)
    assert e_T <= TOL64 and e_G <= TOL64


def test_load_vector_at_sampled_rows(raster_run):
    w, gm, om, n, f0, f1 = raster_run
    F = f1[2]
    R = om.bt["R"].tocsc()
    Rn = R[om.neu]
    lateral_rows = np.nonzero(np.asarray(Rn.sum(axis=0)).ravel() > 0)[0]
    rng = np.random.default_rng(12)
    rows = np.sort(rng.choice(lateral_rows, 40, replace=False))
    sub = Rn[:, rows]
    pts = np.unique(sub.nonzero()[0])                       # NEUMANN points in those rows' support
    sc = w.scan
    _, G = pointsource.field(om.bt["x"][om.neu][pts], sc.xyz, sc.tick, sc.energy, n, sc, w.material)
    flux = -w.material.k * np.einsum("qi,qi->q", G, om.bt["n"][om.neu][pts]) * om.bt["wdS"][om.neu][pts]
    Fr = sub[pts].T @ flux
    e = rel(F[rows], Fr)
    print(f"F rel {e:.2e} at {len(rows)} rows ({len(pts)} points)", flush=True)
    assert e <= TOL64


def test_dirichlet_values_full_projection(raster_run):
    w, gm, om, n, f0, f1 = raster_run
    du = f1[3]
    T_dir, _ = om.boundary_field(n, om.dir)
    wD = om.dirichlet_values(T_dir)
    e = rel(du[om.D], wD)
    print(f"Dirichlet values rel {e:.2e} over {len(om.D)} DOFs", flush=True)
    assert e <= TOL64


def test_theta_step_equation_at_sampled_rows(raster_run):
    w, gm, om, n, f0, f1 = raster_run
    w0, F0 = f0[3], f0[2]
    w1, F1 = f1[3], f1[2]
    rng = np.random.default_rng(13)
    rows = np.sort(rng.choice(om.I, 40, replace=False))
    M, K = iga.assemble_mk(w.patch, w.material, elems=iga.elements_touching(w.patch, rows), rows=rows)
    dt, th = w.scan.dt, 0.5
    lhs = (M[rows] / dt + th * K[rows]) @ w1
    rhs = (M[rows] / dt - (1.0 - th) * K[rows]) @ w0 + th * F1[rows] + (1.0 - th) * F0[rows]
    e = float(np.abs(lhs - rhs).max() / np.abs(rhs).max())
    print(f"theta-step residual rel {e:.2e} at {len(rows)} rows", flush=True)
    assert e <= TOL64
