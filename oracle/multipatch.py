"""Several NURBS patches glued conformingly into one model (the multi-patch
parts of Sec. 3.3; the method of Secs. 2.1-2.4 is unchanged).

Test infrastructure only (see the package docstring).

Patches meet face to face with matching knot vectors and control points
along the shared face, so the union of their spline spaces is continuous
(C0) across the interface: every shared control point is one unknown.  The
caller numbers the control points globally (index_maps[p][A] = global index
of control point A of patch p, equal for the shared ones).  Then
  * M and K (Eqs. 16-17) are the sums of the patches' matrices scattered to
    the global numbering (each element belongs to one patch);
  * the boundary points are the Gauss points of the patch faces that are not
    interfaces (role INTERFACE), with the basis values scattered likewise;
  * the Dirichlet unknowns are the global indices of the patches' Dirichlet
    face layers;
and the load vector, the Dirichlet projection, the theta-scheme and the
reconstruction are those of solver.Model, unchanged.

Reading: the paper shows a multi-patch part (Sec. 3.3) but neither its
geometry nor how its patches are joined; conforming C0 gluing by shared
control points is the plain construction for matching patches.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bspline, iga, pointsource
from .solver import DIRICHLET, NEUMANN, Model

INTERFACE = 3


def _scatter(n_global, gmap):
    """Selection matrix S [n_local, n_global]: S[A, gmap[A]] = 1."""
    n = len(gmap)
    return sp.csr_matrix((np.ones(n), (np.arange(n), np.asarray(gmap))), shape=(n, n_global))


class MultiPatchModel(Model):
    def __init__(self, patches, index_maps, material, scan, theta=0.5, kernel_scale=1.0, path=0):
        self.patches = list(patches)
        self.maps = [np.asarray(g, np.int64) for g in index_maps]
        self.patch = None                      # no single patch: evaluation goes by patch index
        self.mat = material
        self.scan = scan.path(path) if scan.n_paths > 1 or path else scan
        self.theta, self.s = theta, kernel_scale
        self.dt = self.scan.dt
        n = int(max(g.max() for g in self.maps)) + 1
        self.n_dof = n
        S = [_scatter(n, g) for g in self.maps]
        # Eqs. 16-17 patch by patch, scattered to the global numbering
        self.M = sp.csr_matrix((n, n))
        self.K = sp.csr_matrix((n, n))
        for P, Sp in zip(self.patches, S):
            Mp, Kp = iga.assemble_mk(P, material)
            self.M = self.M + Sp.T @ Mp @ Sp
            self.K = self.K + Sp.T @ Kp @ Sp
        self.M, self.K = self.M.tocsr(), self.K.tocsr()
        # boundary points on the faces that are not interfaces
        xs, ns, ws, roles, Rs, self.point_patch = [], [], [], [], [], []
        for p, (P, Sp) in enumerate(zip(self.patches, S)):
            faces = [f for f in range(6) if P.face_role[f] != INTERFACE]
            bt = iga.boundary_tables(P, faces)
            xs.append(bt["x"]); ns.append(bt["n"]); ws.append(bt["wdS"])
            roles.append(np.asarray(P.face_role)[bt["face"]])
            Rs.append(bt["R"] @ Sp)
            self.point_patch.append(np.full(len(bt["wdS"]), p))
        self.bt = {"x": np.concatenate(xs), "n": np.concatenate(ns), "wdS": np.concatenate(ws),
                   "R": sp.vstack(Rs).tocsr()}
        role = np.concatenate(roles)
        self.point_patch = np.concatenate(self.point_patch)
        self.neu = np.nonzero(role == NEUMANN)[0]
        self.dir = np.nonzero(role == DIRICHLET)[0]
        D = [g[iga.dirichlet_dofs(P, f)] for P, g in zip(self.patches, self.maps)
             for f in range(6) if P.face_role[f] == DIRICHLET]
        self.D = np.unique(np.concatenate(D)) if D else np.zeros(0, np.int64)
        mask = np.ones(n, bool)
        mask[self.D] = False
        self.I = np.nonzero(mask)[0]
        if len(self.D):
            Rd = self.bt["R"][self.dir][:, self.D]
            self.M_D = (Rd.T @ sp.diags(self.bt["wdS"][self.dir]) @ Rd).tocsc()
            self._lu_D = spla.splu(self.M_D)
        self.w = np.zeros(n)
        self.F = np.zeros(n)
        self.step = 0
        self.A = (self.M / self.dt + theta * self.K).tocsr()
        self.B = (self.M / self.dt - (1.0 - theta) * self.K).tocsr()
        self._lu = spla.splu(self.A[self.I][:, self.I].tocsc())
        self.A_ID = self.A[self.I][:, self.D].tocsr()

    # -- Eq. 21 on one patch --------------------------------------------------
    def evaluate(self, patch_index, xi, u=None, step=None):
        """T and grad T at parametric points xi [Q, 3] of patch `patch_index`."""
        u = self.u if u is None else u
        step = self.step if step is None else step
        P, g = self.patches[patch_index], self.maps[patch_index]
        w = (u - self.mat.T0)[g]
        x, J, idx, R, dR = bspline.geometry(P, np.atleast_2d(xi))
        uh = self.mat.T0 + np.sum(R * w[idx], axis=1)
        gxi = np.einsum("qlj,ql->qj", dR, w[idx])
        gx = np.einsum("qji,qj->qi", np.linalg.inv(J), gxi)
        sc = self.scan
        Tt, Gt = pointsource.field(x, sc.xyz, sc.tick, sc.energy, step, sc, self.mat, self.s)
        return Tt + uh, Gt + gx, x

    def heat_loss(self, patch_index, face, edge_face, quad=4, u=None, step=None):
        """Net heat-loss rate (Sec. 3.1) along an edge of patch `patch_index`:
        at `quad` Gauss points per element of the edge where its face `face`
        meets its face `edge_face`, q~ = -k grad T~ . n and q^ = -k grad T^ . n
        with n the outward unit normal of `face`, T^ from the global control
        values; the arc-length weights ds and the integrals of |q~ + q^| ds and
        |q~| ds (the diagnostic of solver.Model.heat_loss on that patch)."""
        P, g = self.patches[patch_index], self.maps[patch_index]
        d, de = face // 2, edge_face // 2
        if d == de:
            raise ValueError("the faces must meet along an edge")
        e = 3 - d - de
        t, tw = iga.gauss_1d(P.knots[e], quad)
        xi = np.zeros((len(t), 3))
        xi[:, d] = float(face % 2)
        xi[:, de] = float(edge_face % 2)
        xi[:, e] = t
        x, J, idx, R, dR = bspline.geometry(P, xi)
        ds = np.linalg.norm(J[:, :, e], axis=1) * tw
        a, b = [c for c in range(3) if c != d]
        n = np.cross(J[:, :, a], J[:, :, b])
        n /= np.linalg.norm(n, axis=1)[:, None]
        n *= np.sign(np.einsum("qi,qi->q", n, J[:, :, d]) * (1.0 if face % 2 else -1.0))[:, None]
        u = self.u if u is None else u
        step = self.step if step is None else step
        w = (u - self.mat.T0)[g]
        Gh = np.einsum("qji,qj->qi", np.linalg.inv(J), np.einsum("qlj,ql->qj", dR, w[idx]))
        sc = self.scan
        _, Gt = pointsource.field(x, sc.xyz, sc.tick, sc.energy, step, sc, self.mat, self.s)
        k = self.mat.k
        qt = -k * np.einsum("qi,qi->q", Gt, n)
        qh = -k * np.einsum("qi,qi->q", Gh, n)
        return {"xi": xi, "x": x, "n": n, "ds": ds, "q_tilde": qt, "q_hat": qh,
                "net": float(np.sum(np.abs(qt + qh) * ds)), "tilde": float(np.sum(np.abs(qt) * ds))}

    def locate(self, *args, **kwargs):
        raise NotImplementedError("locate on the patch that holds the point (solver.Model of that patch)")
