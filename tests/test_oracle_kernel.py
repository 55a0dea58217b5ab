"""Pins of the oracle's point-source kernel and superposition (paper Eqs. 7-8)
against the heat equation itself, finite differences, the total energy, the
finite-spot profile at activation, and Rosenthal's moving-source solution."""
import math

import numpy as np
from scipy.integrate import quad

import closed_forms as cf
from oracle import pointsource
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG
ALPHA = MAT.k / (MAT.rho * MAT.cp)
RC = MAT.rho * MAT.cp


def _T(x, src, D, E=1e-4, s=1.0):
    T, G = pointsource.kernel(np.atleast_2d(x), np.atleast_2d(src), np.atleast_1d(D),
                              np.atleast_1d(E), MAT, s)
    return T[:, 0], G[:, 0, :]


def test_kernel_solves_heat_equation():
    """rho c dT/dt = k lap T away from the source (central differences)."""
    src = np.array([0.3e-3, 0.2e-3, 1e-3])
    rng = np.random.default_rng(0)
    for D in (2e-5, 1e-4, 1e-3):
        sig = math.sqrt(2 * ALPHA * D)
        for _ in range(5):
            x = src + rng.normal(size=3) * sig
            ht = D * 1e-3
            hx = sig * 1e-3
            dTdt = (_T(x, src, D + ht)[0] - _T(x, src, D - ht)[0]) / (2 * ht)
            lap = 0.0
            for d in range(3):
                e = np.zeros(3)
                e[d] = hx
                lap += (_T(x + e, src, D)[0] - 2 * _T(x, src, D)[0] + _T(x - e, src, D)[0]) / hx ** 2
            scale = abs(_T(x, src, D)[0]) / D
            assert abs(RC * dTdt - MAT.k * lap) < 1e-4 * RC * scale


def test_gradient_matches_central_differences():
    src = np.array([0.3e-3, 0.2e-3, 1e-3])
    rng = np.random.default_rng(1)
    for D in (1e-5, 3e-4):
        sig = math.sqrt(2 * ALPHA * D)
        x = src + rng.normal(size=(20, 3)) * sig
        _, G = _T(x, src, D)
        h = sig * 1e-5
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fd = (_T(x + e, src, D)[0] - _T(x - e, src, D)[0]) / (2 * h)
            np.testing.assert_allclose(G[:, d], fd, rtol=1e-7, atol=1e-9 * np.abs(G).max())


def test_kernel_integrates_to_energy():
    """int over R^3 of rho c T~_I dV = s E (any time)."""
    E = 1.6e-4
    for s in (1.0, 2.0):
        for D in (6e-6, 1e-4, 2e-3):
            sig = math.sqrt(2 * ALPHA * D)
            f = lambda R: 4 * math.pi * R * R * RC * _T(np.array([R, 0, 0]), np.zeros(3), D, E, s)[0][0]
            tot, _ = quad(f, 0, 40 * sig, limit=200, epsabs=0, epsrel=1e-12)
            assert abs(tot - s * E) < 1e-10 * s * E


def test_profile_at_activation_has_spot_radius():
    """At activation (age 0) the finite-spot shift gives exp(-2 R^2 / r^2)."""
    r = 20e-6
    scan = W.single_track((0, 0, 1e-3), (1e-6, 0, 1e-3), 50.0, 1.0, 1e-5, 10, spot_radius=r)
    assert len(scan.tick) == 1
    # step 1 activates ticks 1..10: age of the single source = 10 - 1 = 9 ticks;
    # use a scan whose source tick equals the step end instead
    scan.tick[:] = 10
    x0 = scan.xyz[0]
    R = np.linspace(0, 3 * r, 13)
    pts = x0[None, :] + np.stack([R, 0 * R, 0 * R], axis=1)
    T, _ = pointsource.field(pts, scan.xyz, scan.tick, scan.energy, 1, scan, MAT)
    np.testing.assert_allclose(T / T[0], np.exp(-2 * R ** 2 / r ** 2), rtol=1e-13, atol=1e-300)
    assert T[0] > 0


def test_causality_on_ticks():
    scan = W.single_track((0, 0, 0), (10e-6, 0, 0), 50.0, 1.0, 1e-5, 10)
    x = np.array([[5e-6, 0, 0]])
    T0, _ = pointsource.field(x, scan.xyz, scan.tick, scan.energy, 0, scan, MAT)
    assert T0[0] == 0.0
    # after step 1 exactly ticks 1..10 are on: the sum equals the 10-source sum
    T1, _ = pointsource.field(x, scan.xyz, scan.tick, scan.energy, 1, scan, MAT)
    a = ALPHA
    D = (10 - scan.tick[:10]) * scan.delta + scan.spot_radius ** 2 / (8 * a)
    Tk, _ = pointsource.kernel(x, scan.xyz[:10], D, scan.energy[:10], MAT)
    assert abs(T1[0] - Tk.sum()) < 1e-14 * T1[0]


def test_superposition_tends_to_rosenthal():
    """A long straight track in the unbounded medium approaches the moving
    point-source solution P/(4 pi k R) exp(-v (xi + R)/(2 alpha))."""
    v, P = 1.0, 80.0
    dt, n_s = 1e-5, 10
    L = 20e-3
    scan = W.single_track((0, 0, 0), (L, 0, 0), P, v, dt, n_s, spot_radius=1e-7)
    step = int(scan.n_steps[0])
    xl = scan.xyz[-1]
    rng = np.random.default_rng(3)
    R = rng.uniform(50e-6, 300e-6, 40)
    dirs = rng.normal(size=(40, 3))
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    pts = xl[None, :] + R[:, None] * dirs
    T, _ = pointsource.field(pts, scan.xyz, scan.tick, scan.energy, step, scan, MAT)
    ref = cf.rosenthal(P, v, MAT.k, ALPHA, pts[:, 0] - xl[0], R)
    np.testing.assert_allclose(T, ref, rtol=1e-4)
