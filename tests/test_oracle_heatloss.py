"""Pins of the oracle's net heat-loss rate along a boundary edge (Sec. 3.1:
q~ + q^ = -k dT/dn on the adiabatic faces, and its line integrals, Tables
3-4): the arc-length weights and outward normals against the exact edge
lengths and normals of the block and of the quarter annulus, the correction
flux of an affine field, the cancellation of a source's flux by its mirror
image across the face, and the shrinking of the net flux under refinement."""
import math
import os

import numpy as np
import pytest

from oracle import pointsource, solver
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG
TOP = 5


def _scan_empty(n_steps=2):
    return W.make_scan([(np.zeros((0, 3)), np.zeros(0, np.int64), np.zeros(0))], 1e-5, 5, n_steps=[n_steps])


def _block():
    return W.block_patch((0.1e-3, -0.2e-3, 0.0), (0.9e-3, 0.3e-3, 0.4e-3), (4, 3, 2), 2)


def _annulus():
    return W.annulus_patch(2e-3, 4e-3, 1e-3, (6, 3, 2), 2)


def test_block_edges_lengths_normals_and_points():
    patch = _block()
    m = solver.Model(patch, MAT, _scan_empty(), assemble=False)
    # face y = lo meets the top along x; face x = hi meets it along y
    for face, length, normal, fixed in ((2, 0.8e-3, (0, -1, 0), (1, -0.2e-3)), (1, 0.5e-3, (1, 0, 0), (0, 0.9e-3)),
                                        (0, 0.5e-3, (-1, 0, 0), (0, 0.1e-3)), (3, 0.8e-3, (0, 1, 0), (1, 0.3e-3))):
        r = m.heat_loss(face, TOP, quad=3)
        assert len(r["ds"]) == 3 * (4 if face in (2, 3) else 3)
        assert abs(r["ds"].sum() - length) <= 1e-15 * length * 10
        np.testing.assert_allclose(r["n"], np.tile(normal, (len(r["ds"]), 1)), atol=1e-14)
        np.testing.assert_allclose(r["x"][:, 2], 0.4e-3, rtol=1e-15)
        np.testing.assert_allclose(r["x"][:, fixed[0]], fixed[1], atol=1e-18)
        assert r["net"] == 0.0 and r["tilde"] == 0.0       # no source, no correction


@pytest.mark.parametrize("face,radius,sign", [(3, 4e-3, 1.0), (2, 2e-3, -1.0)])
def test_annulus_arc_edges_lengths_and_radial_normals(face, radius, sign):
    patch = _annulus()
    m = solver.Model(patch, MAT, _scan_empty(), assemble=False)
    r = m.heat_loss(face, TOP, quad=4)
    x, n = r["x"], r["n"]
    rad = np.hypot(x[:, 0], x[:, 1])
    np.testing.assert_allclose(rad, radius, rtol=1e-14)
    np.testing.assert_allclose(x[:, 2], 1e-3, rtol=1e-14)
    radial = np.stack([x[:, 0] / rad, x[:, 1] / rad, np.zeros_like(rad)], axis=1)
    np.testing.assert_allclose(n, sign * radial, atol=1e-14)
    assert abs(r["ds"].sum() - 0.5 * math.pi * radius) <= 1e-10 * radius


@pytest.mark.parametrize("which", ["block", "annulus"])
def test_affine_correction_has_the_flux_of_its_gradient(which):
    """Control values a.P_A + b reproduce T^ = a.x + b (NURBS reproduce the
    affine functions of the geometry), so q^ = -k a.n at every edge point."""
    patch = _block() if which == "block" else _annulus()
    m = solver.Model(patch, MAT, _scan_empty(), assemble=False)
    a = np.array([3e3, -1.7e3, 2.2e3])
    P = patch.ctrl[..., :3].reshape(-1, 3)
    u = MAT.T0 + 5.0 + P @ a
    for face in (0, 1, 2, 3):
        r = m.heat_loss(face, TOP, quad=3, u=u, step=0)
        np.testing.assert_allclose(r["q_hat"], -MAT.k * (r["n"] @ a), rtol=1e-10, atol=1e-10 * MAT.k * 3e3)
        assert np.all(r["q_tilde"] == 0.0)


def test_mirror_source_cancels_the_source_flux_on_the_face():
    """A source at distance y0 from the face y = lo and its mirror image at
    -y0 have opposite normal derivatives on that face, so the source's q~ at
    the edge points plus the image's flux (formed here from the kernel of
    Eq. 8) vanishes: q~ uses the face's outward normal and the field's
    gradient at the edge points."""
    patch = _block()
    tr = W.single_track((0.3e-3, -0.12e-3, 0.4e-3), (0.7e-3, -0.12e-3, 0.4e-3), 60.0, 1.0, 1e-5, 5)
    m = solver.Model(patch, MAT, tr, assemble=False)
    step = 30
    r = m.heat_loss(2, TOP, quad=4, step=step)
    img = tr.xyz.copy()
    img[:, 1] = 2 * (-0.2e-3) - img[:, 1]
    _, G = pointsource.field(r["x"], img, tr.tick, tr.energy, step, tr, MAT)
    q_img = -MAT.k * np.einsum("qi,qi->q", G, r["n"])
    assert np.abs(r["q_tilde"]).max() > 1e3
    assert np.abs(r["q_tilde"] + q_img).max() <= 1e-12 * np.abs(r["q_tilde"]).max()


def test_net_heat_loss_shrinks_under_refinement():
    """The correction field cancels the source's flux on the adiabatic faces
    better on a finer mesh: the ratio of the integrated |q~ + q^| to the
    integrated |q~| along the top edge of the face nearest the track falls."""
    tr = W.single_track((0.25e-3, 0.1e-3, 0.4e-3), (0.55e-3, 0.1e-3, 0.4e-3), 60.0, 1.0, 1e-5, 5)
    ratios = []
    for n_el in ((4, 3, 3), (8, 6, 6), (16, 12, 12)):
        patch = W.block_patch((0, 0, 0), (0.8e-3, 0.6e-3, 0.4e-3), n_el, 2)
        m = solver.Model(patch, MAT, tr)
        m.advance(20)
        r = m.heat_loss(2, TOP, quad=4)
        ratios.append(r["net"] / r["tilde"])
    print("integrated |q~ + q^| / |q~| under refinement:", ["%.3f" % x for x in ratios], flush=True)
    assert ratios[2] < ratios[1] < ratios[0]


def _paper_rows(table):
    rows = []
    for ln in open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_heat_loss.txt")):
        f = ln.split()
        if f and f[0] == table:
            rows.append(f[1:])
    return rows


@pytest.mark.parametrize("kernel_scale,within", [(2.0, True), (1.0, False)])
def test_single_source_flux_integral_matches_table3(kernel_scale, within):
    """Table 3 prints int|q~ + q^| ds and its percentage of int|q~| ds for
    five meshes; every row implies the same int|q~| ds (the analytical
    field's flux through the top arc, mesh-independent), about 3.52e3 W/m.
    The oracle's kernel flux through the arc of the Table 2 part (16 elements
    along the arc resolve the integrand), Ti-6Al-4V, E = A P dt, 100 um from
    the arc on the 45-degree line, age 1.9e-4 s, is within 5 % of it with the
    half-space factor s = 2 (3.3 % low), and half of it with s = 1."""
    rows = _paper_rows("table3")
    implied = [float(net) / (float(pct) / 100.0) for _, net, pct in rows]
    ref = float(np.mean(implied))
    assert max(implied) - min(implied) <= 0.005 * ref
    w = W.e1((8, 1, 1), W.Options(kernel_scale=kernel_scale))
    m = solver.Model(w.patch, w.material, w.scan, kernel_scale=kernel_scale, assemble=False)
    r = m.heat_loss(2, TOP, quad=8, step=20)
    dev = r["tilde"] / ref - 1.0
    print(f"s = {kernel_scale}: int|q~| ds = {r['tilde']:.1f} W/m, paper {ref:.1f} W/m ({100 * dev:+.1f} %)",
          flush=True)
    assert (abs(dev) <= 0.05) == within


def test_contour_scan_flux_integrals_match_table4():
    """Table 4 implies int|q~| ds along the top arc at t = 2 ms and 3 ms of
    the contour scan (both methods' rows agree to 0.2 %); the oracle's value
    with s = 2 is within 1 % at both times (0.47 % low at 2 ms, 0.001 % at
    3 ms)."""
    rows = _paper_rows("table4")
    w = W.e2((8, 1, 1))
    m = solver.Model(w.patch, w.material, w.scan, kernel_scale=2.0, assemble=False)
    for t in ("2.0e-3", "3.0e-3"):
        implied = [float(net) / (float(pct) / 100.0) for _, tt, net, pct in rows if tt == t]
        ref = float(np.mean(implied))
        assert max(implied) - min(implied) <= 0.005 * ref
        step = int(round(float(t) / w.scan.dt))
        r = m.heat_loss(2, TOP, quad=8, step=step)
        dev = r["tilde"] / ref - 1.0
        print(f"t = {t} s: int|q~| ds = {r['tilde']:.4e} W/m, paper {ref:.4e} W/m ({100 * dev:+.3f} %)", flush=True)
        assert abs(dev) <= 0.01
