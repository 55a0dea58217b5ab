"""Pins of the oracle's multi-patch model (patches glued conformingly, Sec.
3.3's kind of part):

  * a block cut into two patches at x = 1 mm is the same spline space as the
    single patch with a C0 knot (multiplicity p) at that plane: the global
    mass and conductivity matrices, the boundary points, their basis values
    and the whole trajectory of a track that crosses the interface agree
    with the single-patch oracle (already pinned on its own);
  * the constant field is in the kernel of K and 1^T M 1 = rho c_p times
    the part's volume;
  * interface faces carry no boundary points, and shared control points get
    one global index;
  * the heat-loss diagnostic along an edge of each half equals the single
    patch's along the same half of the edge.
"""
import numpy as np
import pytest

from oracle import iga, multipatch, solver
from paper_2511_20432_amd import workloads as W

MAT = W.MAT_CFG
N, D, S, I = W.FACE_NEUMANN, W.FACE_DIRICHLET, W.FACE_SOURCE_PLANE, W.FACE_INTERFACE


def _split_and_single(p=2, n=(2, 2, 2)):
    """Two patches [0,1] and [1,2] mm (x) and the single [0,2] mm patch with
    a p-fold knot at the middle."""
    ky, kz = W.open_uniform_knots(n[1], p), W.open_uniform_knots(n[2], p)
    kx = W.open_uniform_knots(n[0], p)
    inner = [i / (2 * n[0]) for i in range(1, 2 * n[0]) if i != n[0]]
    kx2 = np.sort(np.array([0.0] * (p + 1) + inner + [0.5] * p + [1.0] * (p + 1)))
    h = (1e-3, 0.6e-3, 0.4e-3)
    a = W.block_patch_knots((0, 0, 0), (h[0], h[1], h[2]), (kx, ky, kz), p, (N, I, N, N, D, S))
    b = W.block_patch_knots((h[0], 0, 0), (2 * h[0], h[1], h[2]), (kx, ky, kz), p, (I, N, N, N, D, S))
    one = W.block_patch_knots((0, 0, 0), (2 * h[0], h[1], h[2]), (kx2, ky, kz), p, (N, N, N, N, D, S))
    return [a, b], one


def _track():
    return W.single_track((0.7e-3, 0.1e-3, 0.4e-3), (1.3e-3, 0.1e-3, 0.4e-3), 60.0, 1.0, 1e-5, 5)


def _perm_to_single(maps, patches, one):
    """perm[g] = the single patch's index of global control point g."""
    pos = {tuple(np.round(c[:3] * 1e9).astype(np.int64)): i for i, c in enumerate(one.ctrl.reshape(-1, 4))}
    n = max(m.max() for m in maps) + 1
    perm = np.full(n, -1)
    for P, g in zip(patches, maps):
        for A, c in enumerate(P.ctrl.reshape(-1, 4)):
            perm[g[A]] = pos[tuple(np.round(c[:3] * 1e9).astype(np.int64))]
    assert (perm >= 0).all() and len(np.unique(perm)) == n
    return perm


def test_glue_shares_the_interface_layer():
    patches, one = _split_and_single()
    maps, n = W.glue(patches)
    n0, n1, n2 = patches[0].n_ctrl
    assert n == 2 * patches[0].n_dof - n1 * n2 == one.n_dof
    shared = np.intersect1d(maps[0], maps[1])
    assert len(shared) == n1 * n2
    # the shared ones are the x = 1 mm layer of both
    x = patches[0].ctrl.reshape(-1, 4)[:, 0]
    assert np.allclose(x[np.isin(maps[0], shared)], 1e-3, rtol=0, atol=1e-15)


def test_split_block_matrices_and_points_equal_the_c0_patch():
    patches, one = _split_and_single()
    maps, _ = W.glue(patches)
    perm = _perm_to_single(maps, patches, one)
    mp = multipatch.MultiPatchModel(patches, maps, MAT, _track())
    om = solver.Model(one, MAT, _track())
    Pm = np.zeros((len(perm), len(perm)))
    Pm[np.arange(len(perm)), perm] = 1.0          # (Pm u_single)[g] = u_single[perm[g]]
    for A_mp, A_one in ((mp.M, om.M), (mp.K, om.K)):
        ref = Pm @ A_one.toarray() @ Pm.T
        assert np.abs(A_mp.toarray() - ref).max() <= 1e-13 * np.abs(ref).max()
    # boundary points: the same set (no point on the interface)
    key_mp = np.lexsort(mp.bt["x"].T[::-1])
    key_one = np.lexsort(om.bt["x"].T[::-1])
    np.testing.assert_allclose(mp.bt["x"][key_mp], om.bt["x"][key_one], rtol=0, atol=1e-15)
    np.testing.assert_allclose(mp.bt["n"][key_mp], om.bt["n"][key_one], rtol=0, atol=1e-14)
    np.testing.assert_allclose(mp.bt["wdS"][key_mp], om.bt["wdS"][key_one], rtol=1e-13)
    R_mp = mp.bt["R"][key_mp].toarray()
    R_one = om.bt["R"][key_one].toarray() @ Pm.T
    assert np.abs(R_mp - R_one).max() <= 1e-13
    assert np.array_equal(np.sort(perm[mp.D]), np.sort(om.D))


def test_split_block_trajectory_equals_the_c0_patch():
    patches, one = _split_and_single()
    maps, _ = W.glue(patches)
    perm = _perm_to_single(maps, patches, one)
    mp = multipatch.MultiPatchModel(patches, maps, MAT, _track())
    om = solver.Model(one, MAT, _track())
    mp.advance(30)
    om.advance(30)
    ref = om.w[perm]
    assert np.abs(ref).max() > 0.1
    assert np.abs(mp.w - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.abs(mp.F - om.F[perm]).max() <= 1e-11 * np.abs(om.F).max()
    # evaluation on a patch = evaluation of the single patch at the same point
    xi = np.array([[0.3, 0.4, 0.9], [0.9, 0.5, 1.0]])
    T, G, x = mp.evaluate(1, xi)
    xi1 = xi.copy()
    xi1[:, 0] = 0.5 + 0.5 * xi[:, 0]
    T1, G1, x1 = om.evaluate(xi1)
    np.testing.assert_allclose(x, x1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(T, T1, rtol=1e-12)
    np.testing.assert_allclose(G, G1, rtol=1e-9, atol=1e-9 * np.abs(G1).max())


def test_split_block_heat_loss_equals_the_c0_patch():
    """The heat-loss diagnostic along the top edge of the y- face of each
    half equals the single patch's along the same half of its edge (same
    Gauss points; T^ of the same spline space)."""
    patches, one = _split_and_single()
    maps, _ = W.glue(patches)
    mp = multipatch.MultiPatchModel(patches, maps, MAT, _track())
    om = solver.Model(one, MAT, _track())
    mp.advance(20)
    om.advance(20)
    ref = om.heat_loss(2, 5, quad=3)
    half = len(ref["ds"]) // 2
    for p, sl in ((0, slice(0, half)), (1, slice(half, None))):
        h = mp.heat_loss(p, 2, 5, quad=3)
        np.testing.assert_allclose(h["x"], ref["x"][sl], rtol=0, atol=1e-15)
        np.testing.assert_allclose(h["ds"], ref["ds"][sl], rtol=1e-13)
        scale = np.abs(ref["q_tilde"]).max()
        assert scale > 0
        assert np.abs(h["q_tilde"] - ref["q_tilde"][sl]).max() <= 1e-12 * scale
        assert np.abs(h["q_hat"] - ref["q_hat"][sl]).max() <= 1e-9 * scale


def test_l_part_constant_kernel_volume_and_points():
    w = W.l_part()
    mp = multipatch.MultiPatchModel(w.patches, w.maps, w.material, w.scan)
    one = np.ones(mp.n_dof)
    assert np.abs(mp.K @ one).max() <= 1e-12 * abs(mp.K).max()
    vol = sum(iga.volume(P) for P in w.patches)
    a, b, h = 1e-3, 1e-3, 0.5e-3
    assert vol == pytest.approx(a * a * h + 2 * a * b * h, rel=1e-12)
    assert one @ (mp.M @ one) == pytest.approx(MAT.rho * MAT.cp * vol, rel=1e-12)
    # points on every non-interface face, none inside the part's plan
    q = w.patches[0].quad_face
    per_face = []
    for P in w.patches:
        for f in range(6):
            if P.face_role[f] == I:
                continue
            d = f // 2
            m = [P.n_elem(k) * q for k in range(3) if k != d]
            per_face.append(m[0] * m[1])
    assert len(mp.bt["wdS"]) == sum(per_face)
    x = mp.bt["x"]
    lateral = (x[:, 2] > 1e-12) & (x[:, 2] < h - 1e-12)
    inner = lateral & (x[:, 0] > 1e-12) & (x[:, 1] > 1e-12) & ((x[:, 0] < a - 1e-12) | (x[:, 1] < a - 1e-12))
    on_outer = (np.abs(x[:, 0] - (a + b)) < 1e-12) | (np.abs(x[:, 1] - (a + b)) < 1e-12) | \
               (np.abs(x[:, 0] - a) < 1e-12) | (np.abs(x[:, 1] - a) < 1e-12)
    assert np.all(on_outer[inner])       # lateral points lie on the part's outer sides only
    # Dirichlet unknowns: the bottom layer of every patch, shared ones once
    n_bottom = sum(P.n_ctrl[0] * P.n_ctrl[1] for P in w.patches) - 2 * w.patches[0].n_ctrl[0]
    assert len(mp.D) == n_bottom
