"""Pins of the oracle's load vector (Eq. 18), Dirichlet data (Eq. 11) and
theta-scheme (Eqs. 19-20) against a generalized eigenpair, the discrete and
continuous energy balances, a vanishing-correction case and the exact
image-lattice solution of a rectangular block."""
import math

import numpy as np
import pytest
import scipy.linalg

import closed_forms as cf
from oracle import iga, pointsource, solver
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG
ALPHA = MAT.k / (MAT.rho * MAT.cp)
ALL_NEUMANN = (0, 0, 0, 0, 0, 2)


def _empty_scan(n_steps, dt=1e-5, n_s=5):
    return W.make_scan([(np.zeros((0, 3)), np.zeros(0, np.int64), np.zeros(0))], dt, n_s,
                       n_steps=[n_steps])


@pytest.mark.parametrize("theta", [0.5, 1.0, 0.0])
def test_theta_scheme_amplification_on_eigenpair(theta):
    patch = W.block_patch((0, 0, 0), (0.4e-3, 0.3e-3, 0.2e-3), (3, 2, 2), 2, roles=ALL_NEUMANN)
    m = solver.Model(patch, MAT, _empty_scan(3), theta=theta)
    lam, V = scipy.linalg.eigh(m.K.toarray(), m.M.toarray())
    dt = m.dt
    for j in (1, len(lam) // 2, len(lam) - 1):
        m.u = MAT.T0 + V[:, j]
        m.step = 0
        m.advance(1)
        g = (1 - (1 - theta) * lam[j] * dt) / (1 + theta * lam[j] * dt)
        np.testing.assert_allclose(m.u - MAT.T0, g * V[:, j], atol=1e-9 * np.abs(V[:, j]).max())


def test_discrete_energy_identity_all_neumann():
    """K 1 = 0, so 1^T M (u^n - T0) = dt sum_m (theta F^{m+1} + (1-theta) F^m)."""
    patch = W.block_patch((0, 0, 0), (0.6e-3, 0.4e-3, 0.3e-3), (6, 4, 3), 2, roles=ALL_NEUMANN)
    scan = W.single_track((0.05e-3, 0.05e-3, 0.3e-3), (0.55e-3, 0.05e-3, 0.3e-3), 60.0, 1.0,
                          1e-5, 5)
    m = solver.Model(patch, MAT, scan, theta=0.5)
    one = np.ones(patch.n_dof)
    Fs = [m.F.copy()]
    for _ in range(12):
        m.advance(1)
        Fs.append(m.F.copy())
    lhs = one @ (m.M @ (m.u - MAT.T0))
    rhs = m.dt * sum(0.5 * (one @ Fs[i + 1]) + 0.5 * (one @ Fs[i]) for i in range(12))
    assert abs(rhs) > 0
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)


def test_load_vector_total_equals_box_mass_loss():
    """Sum_A F_A = -k int_{faces} grad T~ . n dS (partition of unity), which for
    a box whose faces (other than the source plane) all take the load is
    -d/dt of the point-source energy inside the box (erf closed form)."""
    size = (1.0e-3, 0.6e-3, 0.5e-3)
    patch = W.block_patch((0, 0, 0), size, (40, 24, 20), 2, roles=ALL_NEUMANN)
    scan = W.single_track((0.2e-3, 0.12e-3, 0.5e-3), (0.8e-3, 0.12e-3, 0.5e-3), 50.0, 1.0,
                          1e-5, 5)
    m = solver.Model(patch, MAT, scan, assemble=False)
    step = 40
    T, G = m.boundary_field(step, m.neu)
    F = m.load_vector(G)
    # closed form: d/dt of sum_i s E_i * fraction_i(D_i), fraction from erf
    now = step * scan.sources_per_step
    act = scan.tick <= now
    D = (now - scan.tick[act]) * scan.delta + scan.spot_radius ** 2 / (8 * ALPHA)
    h = 1e-9
    dmass = 0.0
    for x, E, d in zip(scan.xyz[act], scan.energy[act], D):
        fp = cf.gaussian_box_fraction(x, d + h, ALPHA, (0, 0, 0), size)
        fm = cf.gaussian_box_fraction(x, d - h, ALPHA, (0, 0, 0), size)
        dmass += E * (fp - fm) / (2 * h)
    assert dmass < 0
    assert abs(F.sum() - (-dmass)) < 2e-4 * abs(dmass)


def test_dirichlet_projection_reproduces_trace_functions():
    """The L2 projection is exact on the trace space: Dirichlet data whose
    deviation -T~ from T_c is a bottom-trace spline is returned as its
    coefficients."""
    patch = W.block_patch((0, 0, 0), (0.5e-3, 0.4e-3, 0.3e-3), (3, 3, 2), 2)
    m = solver.Model(patch, MAT, _empty_scan(1), assemble=False)
    rng = np.random.default_rng(4)
    c = rng.normal(size=len(m.D))
    Rd = m.bt["R"][m.dir][:, m.D]
    vals = Rd @ c
    uD = m.dirichlet_values(-vals)
    np.testing.assert_allclose(uD, c, atol=1e-12 * np.abs(c).max())


def test_correction_vanishes_far_from_boundaries():
    """Large block, short central track, short time: the transferred data
    underflow, so T^ stays T_c to rounding."""
    patch = W.block_patch((0, 0, 0), (4e-3, 4e-3, 2e-3), (8, 8, 4), 2)
    scan = W.single_track((1.9e-3, 2e-3, 2e-3), (2.1e-3, 2e-3, 2e-3), 80.0, 1.0, 1e-5, 5)
    m = solver.Model(patch, MAT, scan)
    m.advance(20)
    assert np.abs(m.F).max() < 1e-200
    assert np.abs(m.u - MAT.T0).max() < 1e-9


def _image_correction(src_xyz, D, E, size, pts):
    """Exact T^ - T_c of the block: sum of the non-identity images."""
    out = np.zeros(len(pts))
    for x, d, e in zip(src_xyz, D, E):
        imgs = cf.image_lattice(x, size, n_img=1)
        pos = np.array([p for p, _ in imgs[1:]])
        sg = np.array([s for _, s in imgs[1:]], float)
        T, _ = pointsource.kernel(pts, pos, np.full(len(pos), d), np.full(len(pos), e), MAT)
        out += T @ sg
    return out


@pytest.mark.slow
def test_converges_to_image_lattice_solution():
    """Whole method on a block with adiabatic sides and top and a Dirichlet
    bottom: T^ converges to the image-lattice correction under refinement
    (a track near a vertical edge reflects off two faces)."""
    size = (0.6e-3, 0.6e-3, 0.3e-3)
    errs = []
    for n in (4, 8, 16):
        patch = W.block_patch((0, 0, 0), size, (n, n, max(2, n // 2)), 2)
        scan = W.single_track((0.08e-3, 0.1e-3, 0.3e-3), (0.3e-3, 0.1e-3, 0.3e-3), 60.0, 1.0,
                              1e-5, 5)
        m = solver.Model(patch, MAT, scan)
        m.advance(20)
        rng = np.random.default_rng(5)
        xi = rng.random((300, 3))
        uh, _, x = m.evaluate(xi, correction_only=True)
        now = m.step * scan.sources_per_step
        act = scan.tick <= now
        D = (now - scan.tick[act]) * scan.delta + scan.spot_radius ** 2 / (8 * ALPHA)
        ex = _image_correction(scan.xyz[act], D, scan.energy[act], size, x)
        errs.append(np.abs((uh - MAT.T0) - ex).max() / np.abs(ex).max())
    assert errs[2] < 0.6 * errs[1] < 0.6 * 0.6 * errs[0]
    assert errs[2] < 0.05


def _affine_and_random_cases():
    return [
        ("block", W.block_patch((0, 0, 0), (0.5e-3, 0.4e-3, 0.3e-3), (3, 2, 2), 2)),
        ("annulus", W.annulus_patch(2e-3, 4e-3, 1e-3, n_el=(5, 3, 2), degree=2)),
        ("e1", W.e1_patch()),
    ]


@pytest.mark.parametrize("name,patch", _affine_and_random_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_evaluate_reproduces_affine_fields(name, patch):
    """NURBS reproduce affine functions of the geometry (sum_A R_A = 1 and
    sum_A R_A P_A = x(xi)), so control values u_A = T_c + a.P_A + b give
    T^ = T_c + a.x(xi) + b and grad T^ = a exactly (Eq. 21 with the
    isoparametric gradients of Eq. 14).  A transposed or wrong J^{-1} fails
    on the curved patches, whose Jacobian is not symmetric."""
    m = solver.Model(patch, MAT, _empty_scan(1), assemble=False)
    a = np.array([3.0e4, -1.7e4, 2.2e4])
    b = 4.5
    P = patch.ctrl[..., :3].reshape(-1, 3)
    u = MAT.T0 + P @ a + b
    xi = np.random.default_rng(11).random((60, 3))
    uh, gx, x = m.evaluate(xi, u=u, correction_only=True)
    scale = np.abs(P @ a).max() + b
    np.testing.assert_allclose(uh - MAT.T0, x @ a + b, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(gx, np.broadcast_to(a, gx.shape), rtol=0, atol=1e-9 * np.abs(a).max())


@pytest.mark.parametrize("name,patch", _affine_and_random_cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_evaluate_gradient_matches_physical_differences(name, patch):
    """For random control values the physical gradient returned by evaluate
    predicts the change of T^ between two nearby points from their physical
    offset: grad T^ . (x(xi + h e_j) - x(xi - h e_j)) = T^(xi + h e_j) -
    T^(xi - h e_j) + O(h^3), for each parametric direction j.  The offsets
    come from the geometry map alone, not from the Jacobian."""
    m = solver.Model(patch, MAT, _empty_scan(1), assemble=False)
    u = MAT.T0 + np.random.default_rng(12).normal(size=patch.n_dof)
    xi = 0.05 + 0.9 * np.random.default_rng(13).random((40, 3))
    _, gx, _ = m.evaluate(xi, u=u, correction_only=True)
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        up, _, xp = m.evaluate(xi + e, u=u, correction_only=True)
        um, _, xm = m.evaluate(xi - e, u=u, correction_only=True)
        pred = np.einsum("qi,qi->q", gx, xp - xm)
        np.testing.assert_allclose(pred, up - um, rtol=0, atol=1e-7 * np.abs(up - um).max() + 1e-12)
