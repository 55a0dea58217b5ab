"""Parity of the batched form at full size, in the launch configuration the
benchmark times: the 128 scan strategies of the raster block (64,512
boundary points and 44,555 DOFs per strategy, launch groups of up to 64
paths, tuned tile shape), each put at a seeded mid-scan step with a zeroed
state as the benchmark does, then advanced.  The oracle cannot run the
strategies, so for paths in different launch groups it checks sampled
outputs one by one (Eqs. 7-8, 10-11, 18 and 20 at sampled rows), and the FP32
far-field form is checked against the FP64 form at every boundary point of
every strategy (<= 0.05 K)."""
import numpy as np
import pytest

from oracle import iga, pointsource, solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
WINDOW = 3


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _start_steps(w, window, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(rng.integers(0, max(1, int(L) - window))) for L in w.scan.n_steps]


def _jump(model, steps):
    """Every path at its given step with the zeroed state (checkpoint layout:
    a 32-byte header, then per path its step as int64 and its arrays)."""
    blob = bytearray(model.save())
    per = (len(blob) - 32) // len(steps)
    for p, st in enumerate(steps):
        off = 32 + p * per
        blob[off:off + 8] = int(st).to_bytes(8, "little", signed=True)
    model.load(bytes(blob))


@pytest.fixture(scope="module")
def batch():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg4(seed=0)
    start = _start_steps(w, WINDOW, 0)
    out = {}
    for prec in (W.PRECISION_FP64, W.PRECISION_FP32_FAR):
        m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=prec, tau_near=2e-4))
        _jump(m, start)
        tune = m.autotune(reps=1)
        m.step(WINDOW - 1)
        paths = (0, 63, 64, 127)
        f0 = {p: m.boundary_fields(p) for p in paths}
        m.step(1)
        f1 = {p: m.boundary_fields(p) for p in paths}
        allf = [m.boundary_fields(p) for p in range(w.scan.n_paths)] if prec == W.PRECISION_FP32_FAR else None
        out[prec] = (m, f0, f1, allf, tune)
        print(f"precision {prec}: tuned {tune}, steps of paths 0, 127: {m.get_step(0)}, {m.get_step(127)}",
              flush=True)
    return w, start, out


@pytest.mark.parametrize("p", [0, 63, 64, 127])
def test_batched_path_at_full_size_matches_oracle(batch, p):
    w, start, out = batch
    m, f0, f1, _, _ = out[W.PRECISION_FP64]
    step = start[p] + WINDOW
    assert m.get_step(p) == step
    sc = w.scan.path(p)
    om = solver.Model(w.patch, w.material, sc, assemble=False)
    T, G, F, du = f1[p]
    rng = np.random.default_rng(40 + p)
    q = np.sort(rng.choice(len(T), 300, replace=False))
    Tr, Gr = pointsource.field(om.bt["x"][q], sc.xyz, sc.tick, sc.energy, step, sc, w.material)
    e_T, e_G = rel(T[q], Tr), rel(G[q], Gr)
    # load vector at sampled lateral rows (Eqs. 10, 18)
    Rn = om.bt["R"].tocsc()[om.neu]
    lateral_rows = np.nonzero(np.asarray(Rn.sum(axis=0)).ravel() > 0)[0]
    rows = np.sort(rng.choice(lateral_rows, 20, replace=False))
    sub = Rn[:, rows]
    pts = np.unique(sub.nonzero()[0])
    _, Gp = pointsource.field(om.bt["x"][om.neu][pts], sc.xyz, sc.tick, sc.energy, step, sc, w.material)
    flux = -w.material.k * np.einsum("qi,qi->q", Gp, om.bt["n"][om.neu][pts]) * om.bt["wdS"][om.neu][pts]
    e_F = rel(F[rows], sub[pts].T @ flux)
    # Dirichlet values: the oracle's projection of its own T~ (Eq. 11)
    T_dir, _ = om.boundary_field(step, om.dir)
    e_D = rel(du[om.D], om.dirichlet_values(T_dir))
    # theta-step equation at sampled free rows (Eq. 20)
    w0, F0 = f0[p][3], f0[p][2]
    rws = np.sort(rng.choice(om.I, 20, replace=False))
    M, K = iga.assemble_mk(w.patch, w.material, elems=iga.elements_touching(w.patch, rws), rows=rws)
    dt, th = w.scan.dt, 0.5
    lhs = (M[rws] / dt + th * K[rws]) @ du
    rhs = (M[rws] / dt - (1.0 - th) * K[rws]) @ w0 + th * F[rws] + (1.0 - th) * F0[rws]
    e_S = float(np.abs(lhs - rhs).max() / np.abs(rhs).max())
    print(f"path {p} at step {step}: T~ {e_T:.2e} grad {e_G:.2e} F {e_F:.2e} Dirichlet {e_D:.2e} "
          f"theta-step {e_S:.2e}", flush=True)
    assert max(e_T, e_G, e_F, e_D, e_S) <= TOL64


def test_batched_fp32_far_field_within_005K_at_full_size(batch):
    w, start, out = batch
    m64 = out[W.PRECISION_FP64][0]
    f32 = out[W.PRECISION_FP32_FAR][3]
    worst = 0.0
    for p in range(w.scan.n_paths):
        T64, _, _, u64 = m64.boundary_fields(p)
        T32, _, _, u32 = f32[p]
        worst = max(worst, float(np.abs(T32 - T64).max() + np.abs(u32 - u64).max()))
    print(f"FP32 far field over {w.scan.n_paths} strategies: max |T - T_FP64| <= {worst:.3e} K", flush=True)
    assert worst <= 0.05
