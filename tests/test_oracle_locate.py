"""Pins of the oracle's inverse geometry map and evaluation at physical
points (Eq. 21 at x): the affine block inverts to (x - lo)/(hi - lo) exactly;
on the quarter annulus the radial and height parameters are affine in r and
z, and the angular parameter gives the angle through the closed form of the
rational quadratic Bezier quarter circle; round
trips x(xi(x)) = x on the Table 2 part; points outside every patch are NaN;
the physical-point evaluation equals the parametric one at the located xi."""
import math

import numpy as np

from oracle import solver
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG


def _scan():
    return W.make_scan([(np.zeros((0, 3)), np.zeros(0, np.int64), np.zeros(0))], 1e-5, 5, n_steps=[1])


def test_block_inverse_is_affine():
    lo, hi = np.array([0.1e-3, -0.2e-3, 0.0]), np.array([0.9e-3, 0.3e-3, 0.4e-3])
    patch = W.block_patch(lo, hi, (4, 3, 2), 2)
    m = solver.Model(patch, MAT, _scan(), assemble=False)
    rng = np.random.default_rng(3)
    xi = rng.random((200, 3))
    x = lo + xi * (hi - lo)
    got = m.locate(x)
    np.testing.assert_allclose(got, xi, atol=1e-12)


def test_annulus_inverse_matches_polar_coordinates():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (6, 3, 2), 2)
    m = solver.Model(patch, MAT, _scan(), assemble=False)
    rng = np.random.default_rng(4)
    r = 2e-3 + 2e-3 * rng.random(100)
    phi = 0.5 * math.pi * rng.random(100)
    z = 1e-3 * rng.random(100)
    x = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    xi = m.locate(x)
    np.testing.assert_allclose(xi[:, 1], (r - 2e-3) / 2e-3, atol=1e-12)
    np.testing.assert_allclose(xi[:, 2], z / 1e-3, atol=1e-12)
    from oracle import bspline
    np.testing.assert_allclose(bspline.geometry(patch, xi)[0], x, atol=1e-15)
    # knot insertion keeps the parametrisation of the single rational
    # quadratic Bezier quarter arc P0 = (1, 0), P1 = (1, 1), P2 = (0, 1),
    # weights (1, cos 45, 1): its point at the located parameter has the angle phi
    w = math.cos(math.pi / 4)
    t = xi[:, 0]
    den = (1 - t) ** 2 + 2 * t * (1 - t) * w + t ** 2
    cx = ((1 - t) ** 2 * 1.0 + 2 * t * (1 - t) * w * 1.0 + t ** 2 * 0.0) / den
    cy = ((1 - t) ** 2 * 0.0 + 2 * t * (1 - t) * w * 1.0 + t ** 2 * 1.0) / den
    np.testing.assert_allclose(np.arctan2(cy, cx), phi, atol=1e-12)


def test_round_trip_and_outside_points_on_the_table2_part():
    w = W.e1((3, 2, 2))
    m = solver.Model(w.patch, w.material, w.scan, assemble=False)
    rng = np.random.default_rng(5)
    xi0 = rng.random((150, 3))
    from oracle import bspline
    x = bspline.geometry(w.patch, xi0)[0]
    xi = m.locate(x)
    np.testing.assert_allclose(bspline.geometry(w.patch, xi)[0], x, atol=1e-15)
    np.testing.assert_allclose(xi, xi0, atol=1e-10)
    # inside the removed quarter cylinder, above the part, beside it: outside
    out = np.array([[1.9e-3, 0.1e-3, 1.0e-3], [1.0e-3, 1.0e-3, 2.5e-3], [-0.5e-3, 1.0e-3, 1.0e-3]])
    assert np.isnan(m.locate(out)).all()


def test_physical_evaluation_equals_parametric():
    w = W.cfg1()
    m = solver.Model(w.patch, w.material, w.scan)
    m.advance(12)
    rng = np.random.default_rng(6)
    xi0 = rng.random((40, 3))
    T0, G0, x = m.evaluate(xi0)
    T1, G1, xi = m.evaluate_at(x)
    np.testing.assert_allclose(xi, xi0, atol=1e-11)
    np.testing.assert_allclose(T1, T0, rtol=1e-12)
    np.testing.assert_allclose(G1, G0, rtol=1e-9, atol=1e-9 * np.abs(G0).max())
