"""Pins of the oracle's quadrature, matrices (Eqs. 16-17) and boundary tables
(Eq. 18) against exact volumes and areas, the divergence theorem, the
Kronecker structure of affine blocks (1-D matrices built independently with
scipy's B-splines) and brute-force quadrature."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline, iga
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG
RC = MAT.rho * MAT.cp


def test_gauss_exact_for_polynomials():
    knots = np.array([0, 0, 0, 0.2, 0.7, 1, 1, 1.0])
    for nq in (2, 3, 4):
        x, w = iga.gauss_1d(knots, nq)
        for k in range(2 * nq):
            assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15


def _mats_1d(knots, p, L, nq=12):
    """1-D mass and stiffness matrices of B-splines on [0, L], from scipy's
    BSpline with a high-order Gauss rule per interval (independent of the
    oracle's basis code)."""
    t = np.asarray(knots, float)
    n = len(t) - p - 1
    g, gw = np.polynomial.legendre.leggauss(nq)
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    for s in range(len(t) - 1):
        lo, hi = t[s], t[s + 1]
        if hi <= lo:
            continue
        x = lo + (hi - lo) * (g + 1) / 2
        w = gw * (hi - lo) / 2
        B = np.zeros((n, nq))
        dB = np.zeros((n, nq))
        for i in range(n):
            c = np.zeros(n)
            c[i] = 1
            spl = BSpline(t, c, p)
            B[i] = spl(x)
            dB[i] = spl.derivative()(x)
        M += (B * w) @ B.T * L
        K += (dB * w) @ dB.T / L
    return M, K


@pytest.mark.parametrize("n_el,deg", [((3, 2, 2), 2), ((4, 3, 2), 3), ((2, 2, 3), (1, 2, 3))])
def test_block_matrices_are_kronecker(n_el, deg):
    size = (1.0e-3, 0.7e-3, 0.4e-3)
    patch = W.block_patch((0.1e-3, 0.2e-3, 0.0), np.add((0.1e-3, 0.2e-3, 0.0), size), n_el, deg)
    M, K = iga.assemble_mk(patch, MAT)
    M1 = [None] * 3
    K1 = [None] * 3
    for d in range(3):
        M1[d], K1[d] = _mats_1d(patch.knots[d], patch.degree[d], size[d])
    Mk = RC * np.kron(M1[2], np.kron(M1[1], M1[0]))
    Kk = MAT.k * (np.kron(M1[2], np.kron(M1[1], K1[0])) + np.kron(M1[2], np.kron(K1[1], M1[0]))
                  + np.kron(K1[2], np.kron(M1[1], M1[0])))
    np.testing.assert_allclose(M.toarray(), Mk, atol=1e-14 * np.abs(Mk).max())
    np.testing.assert_allclose(K.toarray(), Kk, atol=1e-12 * np.abs(Kk).max())


def test_mass_total_and_stiffness_kernel_block():
    patch = W.cfg1().patch
    M, K = iga.assemble_mk(patch, MAT)
    one = np.ones(patch.n_dof)
    vol = 2e-3 * 1e-3 * 1e-3
    assert abs(one @ M @ one - RC * vol) < 1e-13 * RC * vol
    assert np.abs(K @ one).max() < 1e-12 * np.abs(K).max()
    assert abs(M - M.T).max() < 1e-15 * abs(M).max()
    assert abs(K - K.T).max() < 1e-15 * abs(K).max()


def test_mass_total_and_stiffness_kernel_annulus():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (12, 6, 3), 2)
    M, K = iga.assemble_mk(patch, MAT)
    one = np.ones(patch.n_dof)
    vol = 3 * math.pi * 1e-9              # (pi/4)(4^2 - 2^2) mm^2 x 1 mm
    # rational geometry: the 3-point rule is not exact; error shrinks fast
    assert abs(one @ M @ one - RC * vol) < 1e-6 * RC * vol
    assert np.abs(K @ one).max() < 1e-11 * np.abs(K).max()
    ev = np.linalg.eigvalsh(M.toarray())
    assert ev.min() > 0


def _brute_mk(patch, nq=14):
    """Brute force: every function on every element, nq^3 Gauss points, basis
    from scipy's BSpline and an independent rational/geometry evaluation."""
    n0, n1, n2 = patch.n_ctrl
    p = patch.degree
    W_ = patch.ctrl[..., 3]
    P = patch.ctrl[..., :3]
    spl = []
    for d in range(3):
        nd = patch.n_ctrl[d]
        fs = []
        for i in range(nd):
            c = np.zeros(nd)
            c[i] = 1
            fs.append(BSpline(patch.knots[d], c, p[d]))
        spl.append(fs)
    g, gw = np.polynomial.legendre.leggauss(nq)
    n = patch.n_dof
    M = np.zeros((n, n))
    K = np.zeros((n, n))
    els = [[(a, b) for a, b in zip(patch.knots[d][:-1], patch.knots[d][1:]) if b > a] for d in range(3)]
    for (l0, h0) in els[0]:
        for (l1, h1) in els[1]:
            for (l2, h2) in els[2]:
                xs = [l + (h - l) * (g + 1) / 2 for l, h in ((l0, h0), (l1, h1), (l2, h2))]
                ws = [gw * (h - l) / 2 for l, h in ((l0, h0), (l1, h1), (l2, h2))]
                V = [np.array([f(xs[d]) for f in spl[d]]) for d in range(3)]      # [n_d, nq]
                dV = [np.array([f.derivative()(xs[d]) for f in spl[d]]) for d in range(3)]
                # tensor basis [a2,a1,a0,q2,q1,q0]
                Nt = np.einsum("ix,jy,kz->kjizyx", V[0], V[1], V[2])
                d0 = np.einsum("ix,jy,kz->kjizyx", dV[0], V[1], V[2])
                d1 = np.einsum("ix,jy,kz->kjizyx", V[0], dV[1], V[2])
                d2 = np.einsum("ix,jy,kz->kjizyx", V[0], V[1], dV[2])
                Wsum = np.einsum("kji,kjizyx->zyx", W_, Nt)
                dW = [np.einsum("kji,kjizyx->zyx", W_, dd) for dd in (d0, d1, d2)]
                R = W_[..., None, None, None] * Nt / Wsum
                dR = [W_[..., None, None, None] * (dd * Wsum - Nt * dw) / Wsum ** 2
                      for dd, dw in zip((d0, d1, d2), dW)]
                R = R.reshape(n, -1)
                dR = np.stack([r.reshape(n, -1) for r in dR], axis=-1)     # [n, Q, 3]
                Pf = P.reshape(n, 3)
                J = np.einsum("nqj,ni->qij", dR, Pf)
                det = np.linalg.det(J)
                Ji = np.linalg.inv(J)
                gx = np.einsum("nqj,qji->nqi", dR, Ji)
                wq = np.einsum("z,y,x->zyx", ws[2], ws[1], ws[0]).ravel() * np.abs(det)
                M += RC * (R * wq) @ R.T
                K += MAT.k * np.einsum("aqi,bqi,q->ab", gx, gx, wq)
    return M, K


def test_brute_force_small_curved_mesh():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (2, 1, 1), 2, quad_vol=(8, 8, 8))
    M, K = iga.assemble_mk(patch, MAT)
    Mb, Kb = _brute_mk(patch)
    np.testing.assert_allclose(M.toarray(), Mb, atol=1e-12 * np.abs(Mb).max())
    np.testing.assert_allclose(K.toarray(), Kb, atol=1e-10 * np.abs(Kb).max())


def test_brute_force_default_rule_close_on_curved_mesh():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (2, 1, 1), 2)
    M, K = iga.assemble_mk(patch, MAT)
    Mb, Kb = _brute_mk(patch)
    assert np.abs(M.toarray() - Mb).max() < 1e-3 * np.abs(Mb).max()
    assert np.abs(K.toarray() - Kb).max() < 1e-2 * np.abs(Kb).max()


def test_boundary_tables_block():
    patch = W.block_patch((0, 0, 0), (2e-3, 1e-3, 0.5e-3), (4, 3, 2), 2)
    bt = iga.boundary_tables(patch)
    areas = {0: 0.5e-6, 1: 0.5e-6, 2: 1e-6, 3: 1e-6, 4: 2e-6, 5: 2e-6}
    normals = {0: (-1, 0, 0), 1: (1, 0, 0), 2: (0, -1, 0), 3: (0, 1, 0), 4: (0, 0, -1), 5: (0, 0, 1)}
    for f in range(6):
        a, b = bt["face_range"][f]
        assert abs(bt["wdS"][a:b].sum() - areas[f]) < 1e-15 * areas[f] * 10
        np.testing.assert_allclose(bt["n"][a:b], np.tile(normals[f], (b - a, 1)), atol=1e-14)
    vol = 2e-3 * 1e-3 * 0.5e-3
    assert abs(np.sum(np.einsum("qi,qi->q", bt["x"], bt["n"]) * bt["wdS"]) - 3 * vol) < 1e-12 * vol
    np.testing.assert_allclose((bt["n"] * bt["wdS"][:, None]).sum(0), 0, atol=1e-20)
    # R rows are the basis at the points: partition of unity, (p+1)^2 non-zeros
    np.testing.assert_allclose(np.asarray(bt["R"].sum(axis=1)).ravel(), 1.0, atol=1e-14)
    assert bt["R"].getnnz(axis=1).max() == 9


def test_boundary_tables_annulus():
    patch = W.annulus_patch(2e-3, 4e-3, 1e-3, (16, 8, 4), 2)
    bt = iga.boundary_tables(patch)
    x, n, w = bt["x"], bt["n"], bt["wdS"]
    mm2 = 1e-6
    area = {0: 2 * mm2, 1: 2 * mm2, 2: math.pi * mm2, 3: 2 * math.pi * mm2,
            4: 3 * math.pi * mm2, 5: 3 * math.pi * mm2}
    for f in range(6):
        a, b = bt["face_range"][f]
        assert abs(w[a:b].sum() - area[f]) < 1e-7 * area[f]
    # arc normals are radial (inward on the inner arc, outward on the outer)
    for f, sgn in ((2, -1), (3, 1)):
        a, b = bt["face_range"][f]
        r = np.hypot(x[a:b, 0], x[a:b, 1])
        ref = sgn * np.stack([x[a:b, 0] / r, x[a:b, 1] / r, 0 * r], axis=1)
        np.testing.assert_allclose(n[a:b], ref, atol=5e-14)
    a, b = bt["face_range"][0]
    np.testing.assert_allclose(n[a:b], np.tile((0, -1, 0), (b - a, 1)), atol=1e-14)
    a, b = bt["face_range"][1]
    np.testing.assert_allclose(n[a:b], np.tile((-1, 0, 0), (b - a, 1)), atol=1e-14)
    a, b = bt["face_range"][5]
    np.testing.assert_allclose(n[a:b], np.tile((0, 0, 1), (b - a, 1)), atol=1e-14)
    vol = 3 * math.pi * 1e-9
    flux = np.sum(np.einsum("qi,qi->q", x, n) * w)
    assert abs(flux - 3 * vol) < 1e-7 * vol
    np.testing.assert_allclose((n * w[:, None]).sum(0), 0, atol=1e-10 * w.sum())


def test_dirichlet_dofs_are_bottom_layer():
    patch = W.block_patch((0, 0, 0), (1e-3, 1e-3, 1e-3), (3, 2, 4), 2)
    D = iga.dirichlet_dofs(patch, 4)
    bt = iga.boundary_tables(patch, faces=[4])
    cols = np.unique(bt["R"].indices)
    np.testing.assert_array_equal(np.sort(D), cols)
