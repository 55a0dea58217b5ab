"""Multi-patch models through the C ABI (sa_mp_*) against the FP64 oracle's
multi-patch model: the three-patch L-shaped part with a track that crosses
both interfaces.

  * FP64: T~ and grad T~ at the boundary points, the load vector and the
    control values after 40 and 150 steps within 1e-9 (normwise), and T,
    grad T at 100 parametric points of each patch (20 on the top face)
    within 1e-9 of the fields' scale, and at physical points found by the
    inverse map; the heat-loss diagnostic along edges of each patch;
  * FP32 far field: within 0.05 K of the oracle over the same steps;
  * a finer L-shaped part (9,360 unknowns) over 60 steps within 1e-9;
  * the additive Schwarz and the Jacobi preconditioners on the same steps;
  * two scan paths in one object, each against the oracle, the second
    bitwise equal to an object that holds it alone;
  * a failed solve leaves the last completed step's state.
"""
import numpy as np
import pytest

from oracle import multipatch
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _models(w, precision=W.PRECISION_FP64):
    from paper_2511_20432_amd import sa_iga
    gm = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, w.scan,
                                W.Options(precision=precision, tau_near=2e-4))
    om = multipatch.MultiPatchModel(w.patches, w.maps, w.material, w.scan)
    return gm, om


def test_l_part_fp64_matches_oracle():
    w = W.l_part()
    gm, om = _models(w)
    info = gm.get_info()
    assert info.n_patches == 3 and info.n_dof == om.n_dof and info.n_bpts == len(om.bt["wdS"])
    assert info.n_dirichlet == len(om.D)
    x, n, wdS = gm.boundary_points()
    assert np.abs(x - om.bt["x"]).max() <= 1e-15 and np.abs(wdS - om.bt["wdS"]).max() <= 1e-13 * wdS.max()
    done = 0
    for s in (40, 150):
        gm.step(s - done)
        om.advance(s - done)
        done = s
        T, G, F, du = gm.boundary_fields()
        Tr, Gr = om.boundary_field(s)
        errs = {"T": rel(T, Tr), "grad": rel(G, Gr), "F": rel(F, om.F), "du": rel(du, om.w)}
        print(f"L part, {info.n_dof} DOFs, step {s}: max |w| {np.abs(om.w).max():.3e} K, worst rel "
              f"{max(errs.values()):.2e}, CG iterations per step {gm.get_info().pcg_iterations / s:.1f}", flush=True)
        assert max(errs.values()) <= TOL, errs
    # T and grad T at 100 parametric points of each patch, 20 on the top
    # face, on the scale of the fields (the control values and the boundary
    # gradients): most random points lie where T^ and T~ are small, and the
    # control values' solve error (~1e-12 of max |w|) grows by 1/h in grad T^
    rng = np.random.default_rng(3)
    scale_T = np.abs(om.w).max()
    scale_G = np.abs(Gr).max()
    for p in range(3):
        xi = rng.uniform(0, 1, (100, 3))
        xi[:20, 2] = 1.0
        T, G = gm.eval_temperature(p, xi)
        Tr_p, Gr_p, _ = om.evaluate(p, xi)
        assert np.abs(T - Tr_p).max() <= TOL * max(scale_T, np.abs(Tr_p - w.material.T0).max())
        assert np.abs(G - Gr_p).max() <= TOL * max(scale_G, np.abs(Gr_p).max())


def test_l_part_physical_points():
    """T and grad T at physical points: each point found in its patch by the
    inverse map (parametric point within 1e-9), the values those of the
    oracle at the parametric point; points in no patch give NaN and -1."""
    w = W.l_part()
    gm, om = _models(w)
    gm.step(50)
    om.advance(50)
    rng = np.random.default_rng(5)
    xs, owners, xis, Trs, Grs = [], [], [], [], []
    for p in range(3):
        xi = rng.uniform(0.02, 0.98, (40, 3))
        xi[:10, 2] = 1.0                   # on the top face
        Tr, Gr, x = om.evaluate(p, xi)
        xs.append(x)
        owners.append(np.full(len(xi), p))
        xis.append(xi)
        Trs.append(Tr)
        Grs.append(Gr)
    x = np.concatenate(xs + [np.array([[1.5e-3, 1.5e-3, 0.25e-3], [-1e-4, 0.5e-3, 0.25e-3]])])
    T, G, patch, xi = gm.eval_temperature_at(x)
    n = len(x) - 2
    Tr, Gr = np.concatenate(Trs), np.concatenate(Grs)
    assert np.array_equal(patch[:n], np.concatenate(owners))
    assert np.abs(xi[:n] - np.concatenate(xis)).max() <= 1e-9
    T0 = w.material.T0
    assert np.abs(T[:n] - Tr).max() <= TOL * np.abs(Tr - T0).max()
    assert np.abs(G[:n] - Gr).max() <= 1e-8 * np.abs(Gr).max()
    # the notch of the L and a point beside the part: in no patch
    assert (patch[n:] == -1).all() and np.isnan(T[n:]).all() and np.isnan(G[n:]).all()


def test_l_part_heat_loss_matches_oracle():
    """The heat-loss diagnostic along the top edges of an outer lateral face
    of each patch against the oracle's.  The edges' fluxes span eleven
    orders (the track starts 0.2 mm from the face x = 2 mm of the arm along
    x), so every edge is judged on the scale of the largest: its largest
    |q| and integral, at 1e-9."""
    w = W.l_part()
    gm, om = _models(w)
    gm.step(80)
    om.advance(80)
    edges = ((0, 2), (1, 1), (2, 3))
    ref = {e: om.heat_loss(e[0], e[1], 5, quad=4) for e in edges}
    qs = max(max(np.abs(r["q_tilde"]).max(), np.abs(r["q_hat"]).max()) for r in ref.values())
    ints = max(max(r["net"], r["tilde"]) for r in ref.values())
    assert qs > 1e3 and ints > 1.0
    for (p, face), r in ref.items():
        g = gm.heat_loss(p, face, 5, quad=4)
        errs = {"q_tilde": np.abs(g["q_tilde"] - r["q_tilde"]).max() / qs,
                "q_hat": np.abs(g["q_hat"] - r["q_hat"]).max() / qs,
                "net": abs(g["net"] - r["net"]) / ints, "tilde": abs(g["tilde"] - r["tilde"]) / ints}
        print(f"patch {p} face {face}: net {g['net']:.6e} (oracle {r['net']:.6e}); worst rel "
              f"{max(errs.values()):.2e}", flush=True)
        assert np.abs(g["x"] - r["x"]).max() <= 1e-15 and np.abs(g["n"] - r["n"]).max() <= 1e-14
        assert np.abs(g["ds"] - r["ds"]).max() <= 1e-13 * r["ds"].max()
        assert max(errs.values()) <= TOL, errs


def test_l_part_fp32_far_within_005K():
    w = W.l_part()
    gm, om = _models(w, W.PRECISION_FP32_FAR)
    om.advance(150)
    gm.step(150)
    T, _, _, du = gm.boundary_fields()
    Tr, _ = om.boundary_field(150)
    e = float(np.abs(T - Tr).max() + np.abs(du - om.w).max())
    print(f"L part FP32 far field, step 150: |dT~| + |dw| = {e:.2e} K", flush=True)
    assert e <= 0.05


def test_finer_l_part_matches_oracle():
    w = W.l_part(n_el=(16, 16, 8))
    gm, om = _models(w)
    gm.step(60)
    om.advance(60)
    _, _, F, du = gm.boundary_fields()
    errs = {"F": rel(F, om.F), "du": rel(du, om.w)}
    print(f"finer L part, {gm.get_info().n_dof} DOFs, step 60: worst rel {max(errs.values()):.2e}", flush=True)
    assert max(errs.values()) <= TOL, errs


def test_l_part_schwarz_and_jacobi_preconditioners_agree():
    """The additive Schwarz preconditioner (each patch's fast-diagonalisation
    solve) and Jacobi give the same trajectory to the solver tolerance, the
    Schwarz solves in far fewer CG iterations."""
    from paper_2511_20432_amd import sa_iga
    w = W.l_part()
    runs = {}
    for name, pc in (("schwarz", W.PRECOND_FD), ("jacobi", W.PRECOND_JACOBI)):
        gm = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, w.scan,
                                    W.Options(tau_near=2e-4, preconditioner=pc))
        gm.step(60)
        info = gm.get_info()
        _, _, F, du = gm.boundary_fields()
        runs[name] = (F, du, info.pcg_iterations / 60, info.dirichlet_iterations / 60)
        print(f"{name}: CG iterations per step {runs[name][2]:.1f}, projection {runs[name][3]:.1f}", flush=True)
    (Fs, us, its, ids), (Fj, uj, itj, idj) = runs["schwarz"], runs["jacobi"]
    assert rel(Fs, Fj) <= 1e-10 and rel(us, uj) <= 1e-10
    assert its <= itj / 3 and ids <= idj / 3


def test_steps_stop_at_the_end_of_the_scan():
    from paper_2511_20432_amd import sa_iga
    w = W.l_part()
    scan = W.make_scan([(w.scan.xyz[:20], w.scan.tick[:20], w.scan.energy[:20])], w.scan.dt,
                       w.scan.sources_per_step, n_steps=[4])
    gm = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, scan)
    gm.step(10)
    assert gm.get_info().step == 4
    with pytest.raises(sa_iga.SaError):
        gm.eval_temperature(3, np.zeros((1, 3)))
    with pytest.raises(sa_iga.SaError):
        gm.eval_temperature(0, np.array([[0.5, 0.5, 1.5]]))


def test_l_part_several_paths():
    """Two scan strategies on the L-shaped part in one object, of different
    lengths (the workload's track, 150 of its 260 steps taken; the track run
    from its other end, 100 steps): each path's fields equal the oracle's run
    of that path alone (1e-9), and path 1's queries equal, bit for bit, those
    of an object that holds path 1 alone (the paths share only the operators
    and the work buffers)."""
    from paper_2511_20432_amd import sa_iga
    w = W.l_part()
    s = w.scan
    back = (s.xyz[::-1][:600], s.tick[:600], s.energy[:600])
    scan = W.make_scan([(s.xyz, s.tick, s.energy), back], s.dt, s.sources_per_step, n_steps=[260, 100])
    alone = W.make_scan([back], s.dt, s.sources_per_step, n_steps=[100])
    opts = W.Options(tau_near=2e-4)
    gm = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, scan, opts)
    g1 = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, alone, opts)
    assert gm.get_info().n_paths == 2 and gm.get_info(1).n_steps == 100
    gm.step(150)
    g1.step(150)
    assert gm.get_info(0).step == 150 and gm.get_info(1).step == 100 and g1.get_info().step == 100
    rng = np.random.default_rng(11)
    xi = rng.uniform(0, 1, (30, 3))
    xi[:10, 2] = 1.0
    for path, steps in ((0, 150), (1, 100)):
        om = multipatch.MultiPatchModel(w.patches, w.maps, w.material, scan, path=path)
        om.advance(steps)
        T, G, F, du = gm.boundary_fields(path)
        Tr, Gr = om.boundary_field(steps)
        errs = {"T": rel(T, Tr), "grad": rel(G, Gr), "F": rel(F, om.F), "du": rel(du, om.w)}
        print(f"path {path}, step {steps}: max |w| {np.abs(om.w).max():.3e} K, worst rel {max(errs.values()):.2e}",
              flush=True)
        assert max(errs.values()) <= TOL, errs
        Tq, Gq = gm.eval_temperature(1, xi, path=path)
        Tq_r, Gq_r, _ = om.evaluate(1, xi)
        assert np.abs(Tq - Tq_r).max() <= TOL * max(np.abs(om.w).max(), np.abs(Tq_r - w.material.T0).max())
        assert np.abs(Gq - Gq_r).max() <= TOL * max(np.abs(Gr).max(), np.abs(Gq_r).max())
    # path 1 of the two-path object = the one-path object, bit for bit
    for a, b in zip(gm.boundary_fields(1), g1.boundary_fields()):
        assert np.array_equal(a, b)
    for a, b in zip(gm.eval_temperature(2, xi, path=1), g1.eval_temperature(2, xi)):
        assert np.array_equal(a, b)
    x = np.array([[0.5e-3, 1.5e-3, 0.5e-3], [1.5e-3, 0.5e-3, 0.4e-3]])
    for a, b in zip(gm.eval_temperature_at(x, path=1), g1.eval_temperature_at(x)):
        assert np.array_equal(a, b)
    h, h1 = gm.heat_loss(2, 3, 5, quad=3, path=1), g1.heat_loss(2, 3, 5, quad=3)
    assert all(np.array_equal(h[k], h1[k]) for k in h)
    info, info1 = gm.get_info(1), g1.get_info()
    assert (info.pcg_iterations, info.dirichlet_iterations) == (info1.pcg_iterations, info1.dirichlet_iterations)
    for bad in (-1, 2):
        with pytest.raises(sa_iga.SaError) as e:
            gm.boundary_fields(bad)
        assert e.value.code == sa_iga.SA_ERANGE


def test_failed_solve_keeps_the_last_completed_step():
    """A CG that cannot reach pcg_rtol (1e-30, below FP64 rounding) within
    pcg_max_iter (8) gives SA_ENOCONV on the first step, and
    the path keeps the state before it: step 0, zero boundary fields (the
    step's source field is not published), F, control values and solver
    statistics."""
    from paper_2511_20432_amd import sa_iga
    w = W.l_part()
    bad = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, w.scan,
                                 W.Options(tau_near=2e-4, pcg_rtol=1e-30, pcg_max_iter=8))
    with pytest.raises(sa_iga.SaError) as e:
        bad.step(1)
    assert e.value.code == sa_iga.SA_ENOCONV
    info = bad.get_info()
    assert info.step == 0 and info.pcg_iterations == 0 and info.dirichlet_iterations == 0
    for a in bad.boundary_fields():
        assert np.array_equal(a, np.zeros_like(a))
