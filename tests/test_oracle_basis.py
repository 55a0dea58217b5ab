"""Pins of the oracle's spline basis and geometry (paper Sec. 2.3, Sec. 3.1
Table 2) against scipy's B-spline routine, partition of unity and exact
circular arcs."""
import math
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline
from paper_2511_20432_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")

KNOTS = [
    (2, [0, 0, 0, 0.25, 0.5, 0.75, 1, 1, 1]),
    (3, [0, 0, 0, 0, 0.1, 0.35, 0.5, 0.9, 1, 1, 1, 1]),
    (2, [0, 0, 0, 0.5, 0.5, 1, 1, 1]),        # the paper's Xi (Sec. 3.1)
    (1, [0, 0, 1, 1]),
    (3, list(W.open_uniform_knots(7, 3))),
]


@pytest.mark.parametrize("p,knots", KNOTS)
def test_basis_matches_scipy(p, knots):
    t = np.array(knots, float)
    n = len(t) - p - 1
    xi = np.concatenate([np.linspace(0, 1, 97), [0.5 - 1e-12, 0.5 + 1e-12, 1.0]])
    N, dN = bspline.basis(t, p, xi)
    for i in range(n):
        c = np.zeros(n)
        c[i] = 1.0
        spl = BSpline(t, c, p, extrapolate=False)
        ref = np.nan_to_num(spl(xi))
        dref = np.nan_to_num(spl.derivative()(xi)) if p > 0 else np.zeros_like(xi)
        # scipy evaluates xi = 1 on the closed last interval as well
        np.testing.assert_allclose(N[:, i], ref, atol=1e-14)
        interior = (xi > 0) & (xi < 1)
        np.testing.assert_allclose(dN[interior, i], dref[interior], atol=1e-10, rtol=1e-12)


@pytest.mark.parametrize("p,knots", KNOTS)
def test_partition_of_unity(p, knots):
    xi = np.linspace(0, 1, 301)
    N, dN = bspline.basis(np.array(knots, float), p, xi)
    np.testing.assert_allclose(N.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dN.sum(axis=1), 0.0, atol=1e-11)
    assert (N >= -1e-15).all()


def test_nurbs_partition_of_unity_and_derivative():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (5, 3, 2), 2)
    rng = np.random.default_rng(1)
    xi = rng.random((50, 3))
    idx, R, dR = bspline.nurbs3(patch, xi)
    np.testing.assert_allclose(R.sum(axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(dR.sum(axis=1), 0.0, atol=1e-11)
    # derivative against central differences of the rational functions
    h = 1e-6
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        ip, Rp, _ = bspline.nurbs3(patch, np.clip(xi + e, 0, 1))
        im, Rm, _ = bspline.nurbs3(patch, np.clip(xi - e, 0, 1))
        ok = (xi[:, j] > 2 * h) & (xi[:, j] < 1 - 2 * h)
        same = np.all(ip == idx, axis=1) & np.all(im == idx, axis=1) & ok
        fd = (Rp[same] - Rm[same]) / (2 * h)
        np.testing.assert_allclose(dR[same, :, j], fd, atol=1e-7)


def test_annulus_arcs_are_exact_circles():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (48, 24, 12), 2)
    rng = np.random.default_rng(2)
    s = rng.random(400)
    for r_face, radius in ((0.0, 2e-3), (1.0, 4e-3)):
        xi = np.stack([s, np.full_like(s, r_face), rng.random(400)], axis=1)
        x, J, _, _, _ = bspline.geometry(patch, xi)
        r = np.hypot(x[:, 0], x[:, 1])
        assert np.max(np.abs(r - radius)) <= 1e-14 * radius * 10
    # the angular span is exactly a quarter turn
    x0, _, _, _, _ = bspline.geometry(patch, np.array([[0, 0.5, 0.5], [1, 0.5, 0.5]]))
    assert abs(math.atan2(x0[0, 1], x0[0, 0])) < 1e-15
    assert abs(math.atan2(x0[1, 1], x0[1, 0]) - math.pi / 2) < 1e-15


def _load_e1_net():
    rows = [list(map(float, ln.split())) for ln in open(os.path.join(GOLD, "e1_top_net.txt"))
            if ln.strip() and not ln.startswith("#")]
    net = np.array([[r[1:4], r[4:7]] for r in rows])
    return net


def test_e1_table2_net_transcribed():
    net = _load_e1_net()
    np.testing.assert_allclose(net, W.E1_TOP_NET_MM, atol=1e-15)


def test_e1_arc_is_circle_with_cos_pi8_weights():
    """Table 2's arc column lies on the circle of radius 1 mm about (2, 0);
    with weights cos(pi/8) at the middle points the NURBS curve is that
    circle exactly (and the straight column stays on the polyline)."""
    patch = W.e1_patch(_load_e1_net())
    s = np.linspace(0, 1, 257)
    xi = np.stack([s, np.zeros_like(s), np.ones_like(s)], axis=1)
    x, _, _, _, _ = bspline.geometry(patch, xi)
    r = np.hypot(x[:, 0] - 2e-3, x[:, 1])
    assert np.max(np.abs(r - 1e-3)) < 1e-17 * 100
    assert np.allclose(x[:, 2], 2e-3)
    xi[:, 1] = 1.0
    xo, _, _, _, _ = bspline.geometry(patch, xi)
    on_poly = (np.abs(xo[:, 0]) < 1e-18) | (np.abs(xo[:, 1] - 2e-3) < 1e-18)
    assert on_poly.all()


def test_paper_energy_per_source():
    vals = {}
    for ln in open(os.path.join(GOLD, "paper_values.txt")):
        if ln.strip() and not ln.startswith("#"):
            k, v = ln.split()
            vals[k] = float(v)
    P_abs = vals["absorptivity"] * vals["power_W"]
    # one source per dt (the paper's discretisation) from the input generator
    scan = W.single_track((0, 0, 0), (1e-4, 0, 0), P_abs, 1.0, vals["dt_s"], 1)
    E = scan.energy[0]
    assert float(f"{E:.3g}") == vals["energy_J_printed"]
