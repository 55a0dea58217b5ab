"""Correction field and time stepping (paper Secs. 2.1-2.4).

Test infrastructure only (see the package docstring).

Per theta-step n -> n+1 (t = (n+1) dt) for one scan path:
  1. T~ and grad T~ at every boundary quadrature point (Eqs. 7-8).
  2. Load vector (Eq. 18 with Eq. 10):
        F_A = sum_{q on NEUMANN faces} R_A(x_q) (-k grad T~_q . n_q) w_q dS_q
  3. Dirichlet data (Eq. 11, enforced on the control variables whose
     functions live on the bottom face): the L2 projection of T_c - T~ on the
     trace space of those functions,
        M_D u_D = sum_{q on DIRICHLET faces} R_A(x_q) (T_c - T~_q) w_q dS_q.
  4. Theta-scheme (Eq. 20):
        (M/dt + theta K) u^{n+1} = (M/dt - (1-theta) K) u^n
                                   + theta F^{n+1} + (1-theta) F^n,
     with the Dirichlet unknowns set to u_D and eliminated (their columns
     move to the right-hand side).  The reduced matrix is constant, so it is
     factorised once by scipy's sparse LU (library primitive).
  5. T = T~ + T^ (Eq. 21) for evaluation.
  6. Evaluation at physical points: the parametric point of x is the root
     of x(xi) = x (Newton's method on the geometry map from the nearest
     element centre, kept in [0,1]^3); points not reached are outside.
  7. Net heat-loss rate along a boundary curve (Sec. 3.1, the diagnostic of
     the adiabatic condition): q~ + q^ = -k dT/dn = -k (grad T~ + grad T^) . n
     at Gauss points of the edge where a face meets a neighbouring face, with
     n the outward unit normal of the first face, and the line integrals of
     |q~ + q^| and |q~| over the edge.

Initial state: u^0 = T_c (T^(x, 0) = T_c, and T~(x, 0) = 0), F^0 = 0.

The state is carried as w = u - T_c.  Eqs. 9-11 are linear and the constant
T_c solves them with zero data (K 1 = 0, the projection of the constant
T_c is T_c 1), so w obeys the same theta-scheme with Dirichlet data
-T~ and w^0 = 0; u = T_c + w.  This keeps the T_c offset out of the
rounding of small corrections.

Readings: Dirichlet values by L2 projection (the paper names no method);
SOURCE_PLANE faces take no load (the kernel is adiabatic on the plane that
holds the sources); with no Dirichlet face the problem is pure Neumann.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bspline, iga, pointsource

NEUMANN, DIRICHLET, SOURCE_PLANE = 0, 1, 2


class Model:
    def __init__(self, patch, material, scan, theta=0.5, kernel_scale=1.0, path=0,
                 assemble=True):
        self.patch, self.mat = patch, material
        self.scan = scan.path(path) if scan.n_paths > 1 or path else scan
        self.theta, self.s = theta, kernel_scale
        self.dt = self.scan.dt
        self.bt = iga.boundary_tables(patch)
        face = self.bt["face"]
        role = np.asarray(patch.face_role)[face]
        self.neu = np.nonzero(role == NEUMANN)[0]
        self.dir = np.nonzero(role == DIRICHLET)[0]
        dfaces = [f for f in range(6) if patch.face_role[f] == DIRICHLET]
        D = np.unique(np.concatenate([iga.dirichlet_dofs(patch, f) for f in dfaces])) \
            if dfaces else np.zeros(0, int)
        self.D = D
        mask = np.ones(patch.n_dof, bool)
        mask[D] = False
        self.I = np.nonzero(mask)[0]
        R = self.bt["R"]
        if len(D):
            Rd = R[self.dir][:, D]
            self.M_D = (Rd.T @ sp.diags(self.bt["wdS"][self.dir]) @ Rd).tocsc()
            self._lu_D = spla.splu(self.M_D)
        self.w = np.zeros(patch.n_dof)
        self.F = np.zeros(patch.n_dof)
        self.step = 0
        if assemble:
            self.M, self.K = iga.assemble_mk(patch, material)
            self.A = (self.M / self.dt + theta * self.K).tocsr()
            self.B = (self.M / self.dt - (1.0 - theta) * self.K).tocsr()
            self._lu = spla.splu(self.A[self.I][:, self.I].tocsc())
            self.A_ID = self.A[self.I][:, self.D].tocsr()

    # -- Eqs. 7-8 at the boundary points --------------------------------------
    def boundary_field(self, step, which=None):
        x = self.bt["x"] if which is None else self.bt["x"][which]
        sc = self.scan
        return pointsource.field(x, sc.xyz, sc.tick, sc.energy, step, sc, self.mat, self.s)

    # -- Eq. 18 with Eq. 10 ---------------------------------------------------
    def load_vector(self, G_neu):
        q = -self.mat.k * np.einsum("qi,qi->q", G_neu, self.bt["n"][self.neu]) \
            * self.bt["wdS"][self.neu]
        return self.bt["R"][self.neu].T @ q

    @property
    def u(self):
        """Control values of T^."""
        return self.mat.T0 + self.w

    @u.setter
    def u(self, value):
        self.w = np.asarray(value, float) - self.mat.T0

    # -- Eq. 11 by L2 projection ----------------------------------------------
    def dirichlet_values(self, T_dir):
        """Projection of T_c - T~ minus T_c (the deviation of u_D from T_c)."""
        if len(self.D) == 0:
            return np.zeros(0)
        Rd = self.bt["R"][self.dir][:, self.D]
        b = Rd.T @ ((-T_dir) * self.bt["wdS"][self.dir])
        return self._lu_D.solve(b)

    # -- Eq. 20 ---------------------------------------------------------------
    def advance(self, n=1):
        for _ in range(n):
            s1 = self.step + 1
            idx = np.concatenate([self.neu, self.dir])
            T, G = self.boundary_field(s1, idx)
            nn = len(self.neu)
            F1 = self.load_vector(G[:nn])
            wD = self.dirichlet_values(T[nn:])
            rhs = self.B @ self.w + self.theta * F1 + (1.0 - self.theta) * self.F
            w1 = np.empty_like(self.w)
            w1[self.D] = wD
            r_I = rhs[self.I] - self.A_ID @ wD
            w1[self.I] = self._lu.solve(r_I)
            self.w, self.F, self.step = w1, F1, s1
        return self

    # -- Eq. 21 ---------------------------------------------------------------
    def evaluate(self, xi, u=None, step=None, correction_only=False):
        """T and grad T at parametric points xi [Q, 3] (or only the
        correction T^ and its gradient with correction_only)."""
        u = self.u if u is None else u
        step = self.step if step is None else step
        w = u - self.mat.T0
        x, J, idx, R, dR = bspline.geometry(self.patch, np.atleast_2d(xi))
        uh = self.mat.T0 + np.sum(R * w[idx], axis=1)
        gxi = np.einsum("qlj,ql->qj", dR, w[idx])
        gx = np.einsum("qji,qj->qi", np.linalg.inv(J), gxi)
        if correction_only:
            return uh, gx, x
        sc = self.scan
        Tt, Gt = pointsource.field(x, sc.xyz, sc.tick, sc.energy, step, sc, self.mat, self.s)
        return Tt + uh, Gt + gx, x

    # -- Sec. 3.1: net heat-loss rate along an edge of a face ----------------
    def heat_loss(self, face, edge_face, quad=4, u=None, step=None):
        """q~ = -k grad T~ . n and q^ = -k grad T^ . n at `quad` Gauss points
        per element of the edge where face `face` meets face `edge_face`,
        n the outward unit normal of `face`; with the arc-length weights ds
        and the integrals of |q~ + q^| ds and |q~| ds."""
        d, e_d = face // 2, edge_face // 2
        if d == e_d:
            raise ValueError("the faces must meet along an edge")
        e = 3 - d - e_d                                  # parametric direction along the edge
        t, tw = iga.gauss_1d(self.patch.knots[e], quad)
        xi = np.zeros((len(t), 3))
        xi[:, d] = float(face % 2)
        xi[:, e_d] = float(edge_face % 2)
        xi[:, e] = t
        x, J, _, _, _ = bspline.geometry(self.patch, xi)
        ds = np.linalg.norm(J[:, :, e], axis=1) * tw
        # outward normal: cross product of the face's tangents, oriented so
        # that it points along the parametric direction leaving the patch
        a, b = [c for c in range(3) if c != d]
        n = np.cross(J[:, :, a], J[:, :, b])
        n /= np.linalg.norm(n, axis=1)[:, None]
        out = 1.0 if face % 2 else -1.0
        n *= np.sign(np.einsum("qi,qi->q", n, J[:, :, d]) * out)[:, None]
        step = self.step if step is None else step
        sc = self.scan
        _, Gt = pointsource.field(x, sc.xyz, sc.tick, sc.energy, step, sc, self.mat, self.s)
        _, Gh, _ = self.evaluate(xi, u=u, step=step, correction_only=True)
        k = self.mat.k
        qt = -k * np.einsum("qi,qi->q", Gt, n)
        qh = -k * np.einsum("qi,qi->q", Gh, n)
        return {"xi": xi, "x": x, "n": n, "ds": ds, "q_tilde": qt, "q_hat": qh,
                "net": float(np.sum(np.abs(qt + qh) * ds)), "tilde": float(np.sum(np.abs(qt) * ds))}

    # -- inverse of the geometry map and evaluation at physical points -------
    def locate(self, x, tol=1e-13, iters=60):
        """Parametric points xi [Q, 3] with x(xi) = x [Q, 3]; NaN where the
        Newton iteration from the nearest element centre does not reach x
        (the point lies outside the patch)."""
        x = np.atleast_2d(np.asarray(x, float))
        ctr = []
        for e2 in bspline.elements(self.patch.knots[2]):
            for e1 in bspline.elements(self.patch.knots[1]):
                for e0 in bspline.elements(self.patch.knots[0]):
                    ctr.append([0.5 * (e0[0] + e0[1]), 0.5 * (e1[0] + e1[1]), 0.5 * (e2[0] + e2[1])])
        ctr = np.array(ctr)
        xc = bspline.geometry(self.patch, ctr)[0]
        P = self.patch.ctrl[..., :3].reshape(-1, 3)
        ext = np.abs(P - 0.5 * (P.min(axis=0) + P.max(axis=0))).max()
        d2 = ((x[:, None, :] - xc[None, :, :]) ** 2).sum(axis=-1)
        xi = ctr[np.argmin(d2, axis=1)].copy()
        done = np.zeros(len(x), bool)
        for _ in range(iters):
            xx, J, _, _, _ = bspline.geometry(self.patch, xi)
            r = x - xx
            done = np.linalg.norm(r, axis=1) <= tol * ext
            if done.all():
                break
            step = np.linalg.solve(J, r[:, :, None])[:, :, 0]
            xi = np.where(done[:, None], xi, np.clip(xi + step, 0.0, 1.0))
        xi[~done] = np.nan
        return xi

    def evaluate_at(self, x, u=None, step=None):
        """T and grad T at physical points x [Q, 3] (NaN outside the patch)."""
        xi = self.locate(x)
        ok = ~np.isnan(xi[:, 0])
        T = np.full(len(xi), np.nan)
        G = np.full((len(xi), 3), np.nan)
        if ok.any():
            T[ok], G[ok], _ = self.evaluate(xi[ok], u=u, step=step)
        return T, G, xi
