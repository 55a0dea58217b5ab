"""Isogeometric discretisation of the correction field (paper Sec. 2.3).

Test infrastructure only (see the package docstring).

  * Gauss-Legendre rules on every non-empty knot interval (numpy's leggauss
    is the library primitive for the 1-D rule).
  * Mass and conductivity matrices (Eqs. 16-17):
        M_AB = int rho c_p R_A R_B |det J| dxi
        K_AB = int k (grad_x R_A . grad_x R_B) |det J| dxi
    with grad_x R = J^{-T} grad_xi R and J = dx/dxi (Eq. 14).
  * Boundary quadrature tables for the surface integral of Eq. 18 on every
    parametric face: points x_q, outward unit normals n_q and weights
    w_q dS_q, plus the values R_A(x_q).

Readings (the paper does not state them):
  * volume rule: quad_vol points per direction (p+1 unless the patch says
    otherwise); face rule: quad_face x quad_face per face element;
  * outward normal n = +-(t_a x t_b)/|t_a x t_b| with t_a, t_b the tangents
    along the two in-face parametric directions (a < b); the sign makes
    n . dx/dxi_d negative on the face xi_d = 0 and positive on xi_d = 1;
  * order of boundary points: faces 0..5 = (xi0=0, xi0=1, xi1=0, xi1=1,
    xi2=0, xi2=1); on each face a row-major grid of points over the
    in-face directions (a, b), a fastest, each direction ordered by element
    then Gauss point.  DOF index A = a0 + n0*(a1 + n1*a2).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import bspline


def gauss_1d(knots, nq):
    """Gauss points and weights on every element of one knot vector.

    Returns (xi [n_el*nq], w [n_el*nq]) ordered by element then point."""
    g, gw = np.polynomial.legendre.leggauss(nq)
    xs, ws = [], []
    for lo, hi, _ in bspline.elements(knots):
        xs.append(lo + (hi - lo) * (g + 1.0) / 2.0)
        ws.append(gw * (hi - lo) / 2.0)
    return np.concatenate(xs), np.concatenate(ws)


def _element_points(patch, e):
    """Tensor Gauss points of element e = (e0, e1, e2): xi [Q, 3], w [Q]."""
    pts, wts = [], []
    for d in range(3):
        lo, hi, _ = bspline.elements(patch.knots[d])[e[d]]
        g, gw = np.polynomial.legendre.leggauss(patch.quad_vol[d])
        pts.append(lo + (hi - lo) * (g + 1.0) / 2.0)
        wts.append(gw * (hi - lo) / 2.0)
    X2, X1, X0 = np.meshgrid(pts[2], pts[1], pts[0], indexing="ij")
    W2, W1, W0 = np.meshgrid(wts[2], wts[1], wts[0], indexing="ij")
    xi = np.stack([X0.ravel(), X1.ravel(), X2.ravel()], axis=1)
    return xi, (W0 * W1 * W2).ravel()


def all_elements(patch):
    ne = [patch.n_elem(d) for d in range(3)]
    return [(e0, e1, e2) for e2 in range(ne[2]) for e1 in range(ne[1]) for e0 in range(ne[0])]


def elements_touching(patch, dofs):
    """Elements whose support intersects the given DOFs (for row subsets)."""
    n0, n1, _ = patch.n_ctrl
    p = patch.degree
    spans = [[s for _, _, s in bspline.elements(patch.knots[d])] for d in range(3)]
    out = set()
    for A in np.atleast_1d(dofs):
        a = (A % n0, (A // n0) % n1, A // (n0 * n1))
        cand = []
        for d in range(3):
            # function a_d is non-zero on spans a_d .. a_d + p
            cand.append([i for i, s in enumerate(spans[d]) if a[d] <= s <= a[d] + p[d]])
        for e2 in cand[2]:
            for e1 in cand[1]:
                for e0 in cand[0]:
                    out.add((e0, e1, e2))
    return sorted(out, key=lambda e: (e[2], e[1], e[0]))


def assemble_mk(patch, material, elems=None, rows=None, chunk=512):
    """Mass and conductivity matrices, Eqs. 16-17, as scipy CSR.

    elems: elements to integrate (default all).  rows: keep only these rows
    (the others are zero); pass elements_touching(patch, rows) as elems to
    get exact rows cheaply on big meshes."""
    n = patch.n_dof
    if elems is None:
        elems = all_elements(patch)
    rc = material.rho * material.cp
    keep = None
    if rows is not None:
        keep = np.zeros(n, bool)
        keep[np.asarray(rows)] = True
    Ms, Ks = sp.csr_matrix((n, n)), sp.csr_matrix((n, n))
    for c0 in range(0, len(elems), chunk):
        I, Jc, Mv, Kv = [], [], [], []
        for e in elems[c0:c0 + chunk]:
            xi, wq = _element_points(patch, e)
            x, J, idx, R, dR = bspline.geometry(patch, xi)
            detJ = np.linalg.det(J)
            Jinv = np.linalg.inv(J)
            # grad_x R_A = J^{-T} grad_xi R_A  ->  g[q, l, i] = sum_j dR[q,l,j] Jinv[q,j,i]
            g = np.einsum("qlj,qji->qli", dR, Jinv)
            dv = wq * np.abs(detJ)
            Me = rc * np.einsum("q,qa,qb->ab", dv, R, R)
            Ke = material.k * np.einsum("q,qai,qbi->ab", dv, g, g)
            ids = idx[0]            # same local functions at all points of an element
            I.append(np.repeat(ids, len(ids)))
            Jc.append(np.tile(ids, len(ids)))
            Mv.append(Me.ravel())
            Kv.append(Ke.ravel())
        I = np.concatenate(I)
        Jc = np.concatenate(Jc)
        Mv = np.concatenate(Mv)
        Kv = np.concatenate(Kv)
        if keep is not None:
            m = keep[I]
            I, Jc, Mv, Kv = I[m], Jc[m], Mv[m], Kv[m]
        Ms = Ms + sp.csr_matrix((Mv, (I, Jc)), shape=(n, n))
        Ks = Ks + sp.csr_matrix((Kv, (I, Jc)), shape=(n, n))
    return Ms.tocsr(), Ks.tocsr()


def face_points_param(patch, f):
    """Parametric Gauss points of face f in the canonical order, with the
    parametric (in-face) weights.  Returns xi [Q, 3], w [Q]."""
    d, side = divmod(f, 2)
    a, b = [k for k in range(3) if k != d]
    nq = patch.quad_face
    xa, wa = gauss_1d(patch.knots[a], nq)
    xb, wb = gauss_1d(patch.knots[b], nq)
    XB, XA = np.meshgrid(xb, xa, indexing="ij")          # a fastest
    WB, WA = np.meshgrid(wb, wa, indexing="ij")
    xi = np.zeros((XA.size, 3))
    xi[:, a] = XA.ravel()
    xi[:, b] = XB.ravel()
    xi[:, d] = float(side)
    return xi, (WA * WB).ravel()


def boundary_tables(patch, faces=range(6)):
    """Quadrature tables of the six parametric faces.

    Returns a dict with x [Q,3], n [Q,3], wdS [Q], face [Q] (int),
    R (scipy CSR [Q, n_dof]) = basis values at the points, and the slices
    face_range[f] = (start, stop)."""
    xs, ns, ws, fs, Rs, rng = [], [], [], [], [], {}
    start = 0
    for f in faces:
        d, side = divmod(f, 2)
        a, b = [k for k in range(3) if k != d]
        xi, wp = face_points_param(patch, f)
        x, J, idx, R, dR = bspline.geometry(patch, xi)
        ta, tb, td = J[:, :, a], J[:, :, b], J[:, :, d]
        c = np.cross(ta, tb)
        dS = np.linalg.norm(c, axis=1)
        sgn = np.sign(np.einsum("qi,qi->q", c, td)) * (1.0 if side == 1 else -1.0)
        n = c / dS[:, None] * sgn[:, None]
        Q = len(wp)
        rows = np.repeat(np.arange(Q), idx.shape[1])
        Rm = sp.csr_matrix((R.ravel(), (rows, idx.ravel())), shape=(Q, patch.n_dof))
        Rm.eliminate_zeros()
        xs.append(x); ns.append(n); ws.append(wp * dS); fs.append(np.full(Q, f))
        Rs.append(Rm)
        rng[f] = (start, start + Q)
        start += Q
    return {"x": np.concatenate(xs), "n": np.concatenate(ns), "wdS": np.concatenate(ws),
            "face": np.concatenate(fs), "R": sp.vstack(Rs).tocsr(), "face_range": rng}


def dirichlet_dofs(patch, face=4):
    """Control variables whose functions are non-zero on face `face` (for an
    open knot vector: the first or last layer of control points)."""
    n0, n1, n2 = patch.n_ctrl
    d, side = divmod(face, 2)
    A = np.arange(patch.n_dof)
    a = [A % n0, (A // n0) % n1, A // (n0 * n1)]
    last = (n0, n1, n2)[d] - 1
    return A[a[d] == (last if side else 0)]


def volume(patch):
    """Volume of the patch by the volume quadrature rule."""
    tot = 0.0
    for e in all_elements(patch):
        xi, wq = _element_points(patch, e)
        _, J, _, _, _ = bspline.geometry(patch, xi)
        tot += np.sum(wq * np.abs(np.linalg.det(J)))
    return tot
