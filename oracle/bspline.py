"""B-spline and NURBS basis functions (paper Sec. 2.3, "Isogeometric
discretization": the unknown and the geometry are expanded in B-spline or
NURBS functions of order p on the knot vectors of the parametric domain).

Test infrastructure only (see the package docstring).

The B-splines follow the Cox-de Boor recursion written out over the whole
knot vector (every function, every point), with the convention 0/0 = 0:

    N_{i,0}(xi) = 1 if t_i <= xi < t_{i+1} else 0
    N_{i,q}(xi) = (xi - t_i)/(t_{i+q} - t_i) N_{i,q-1}(xi)
                + (t_{i+q+1} - xi)/(t_{i+q+1} - t_{i+1}) N_{i+1,q-1}(xi)
    N'_{i,q}(xi) = q/(t_{i+q} - t_i) N_{i,q-1}(xi)
                 - q/(t_{i+q+1} - t_{i+1}) N_{i+1,q-1}(xi)

At the right end of an open knot vector (xi = t_last) the last non-empty
interval is taken as closed, so the basis stays a partition of unity there.

NURBS functions are R_A = w_A N_A / sum_B w_B N_B with quotient-rule
derivatives (tensor-product N_A in three dimensions).
"""
from __future__ import annotations

import numpy as np


def _safe_div(a, b):
    out = np.zeros(np.broadcast(a, b).shape)
    nz = b != 0
    np.divide(a, b, out=out, where=np.broadcast_to(nz, out.shape))
    return out


def basis(knots, p, xi):
    """All n = len(knots) - p - 1 B-splines of degree p and their first
    derivatives at the points xi.  Returns (N, dN), each [len(xi), n]."""
    t = np.asarray(knots, float)
    xi = np.atleast_1d(np.asarray(xi, float))
    m = len(t) - 1                       # number of intervals
    # degree 0
    N = ((t[None, :-1] <= xi[:, None]) & (xi[:, None] < t[None, 1:])).astype(float)
    last = np.max(np.nonzero(t[1:] > t[:-1])[0])      # last non-empty interval
    at_end = xi >= t[-1]
    N[at_end, :] = 0.0
    N[at_end, last] = 1.0
    dN = np.zeros_like(N)
    for q in range(1, p + 1):
        n_q = m - q
        left_den = t[q:q + n_q] - t[:n_q]                 # t_{i+q} - t_i
        right_den = t[q + 1:q + 1 + n_q] - t[1:1 + n_q]   # t_{i+q+1} - t_{i+1}
        a = _safe_div(xi[:, None] - t[None, :n_q], left_den[None, :])
        b = _safe_div(t[None, q + 1:q + 1 + n_q] - xi[:, None], right_den[None, :])
        da = _safe_div(np.full((1, n_q), float(q)), left_den[None, :])
        db = _safe_div(np.full((1, n_q), float(q)), right_den[None, :])
        Nlo, Nhi = N[:, :n_q], N[:, 1:n_q + 1]
        dN = da * Nlo - db * Nhi
        N = a * Nlo + b * Nhi
    return N, dN


def span_of(knots, p, xi):
    """Index s of the knot interval [t_s, t_{s+1}) holding xi (p <= s <= n-1);
    the basis functions s-p .. s are the only ones that can be non-zero."""
    t = np.asarray(knots, float)
    n = len(t) - p - 1
    s = np.searchsorted(t, xi, side="right") - 1
    return np.clip(s, p, n - 1)


def elements(knots):
    """Non-empty knot intervals (the elements): list of (t_lo, t_hi, span)."""
    t = np.asarray(knots, float)
    return [(t[s], t[s + 1], s) for s in range(len(t) - 1) if t[s + 1] > t[s]]


def nurbs3(patch, xi):
    """Trivariate NURBS functions at parametric points xi [Q, 3].

    Returns (idx, R, dR): idx [Q, L] global indices A = a0 + n0*(a1 + n1*a2)
    of the L = prod(p_d + 1) functions that can be non-zero, R [Q, L] their
    values and dR [Q, L, 3] their parametric derivatives dR/dxi_j.
    """
    xi = np.atleast_2d(np.asarray(xi, float))
    Q = xi.shape[0]
    n0, n1, n2 = patch.n_ctrl
    p = patch.degree
    loc_idx, loc_N, loc_dN = [], [], []
    for d in range(3):
        N, dN = basis(patch.knots[d], p[d], xi[:, d])
        s = span_of(patch.knots[d], p[d], xi[:, d])
        ids = s[:, None] - p[d] + np.arange(p[d] + 1)[None, :]
        loc_idx.append(ids)
        loc_N.append(np.take_along_axis(N, ids, axis=1))
        loc_dN.append(np.take_along_axis(dN, ids, axis=1))
    i0, i1, i2 = loc_idx
    idx = (i0[:, None, None, :] + n0 * (i1[:, None, :, None] + n1 * i2[:, :, None, None]))
    B = loc_N[2][:, :, None, None] * loc_N[1][:, None, :, None] * loc_N[0][:, None, None, :]
    dB0 = loc_N[2][:, :, None, None] * loc_N[1][:, None, :, None] * loc_dN[0][:, None, None, :]
    dB1 = loc_N[2][:, :, None, None] * loc_dN[1][:, None, :, None] * loc_N[0][:, None, None, :]
    dB2 = loc_dN[2][:, :, None, None] * loc_N[1][:, None, :, None] * loc_N[0][:, None, None, :]
    idx = idx.reshape(Q, -1)
    B = B.reshape(Q, -1)
    dB = np.stack([dB0.reshape(Q, -1), dB1.reshape(Q, -1), dB2.reshape(Q, -1)], axis=-1)
    w = patch.ctrl[..., 3].reshape(-1)[idx]                      # [Q, L]
    W = np.sum(w * B, axis=1)                                    # [Q]
    dW = np.einsum("ql,qlj->qj", w, dB)                          # [Q, 3]
    R = w * B / W[:, None]
    dR = w[:, :, None] * (dB * W[:, None, None] - B[:, :, None] * dW[:, None, :]) \
        / (W[:, None, None] ** 2)
    return idx, R, dR


def geometry(patch, xi):
    """Point x(xi), Jacobian J[i, j] = dx_i/dxi_j, and the basis (idx, R, dR)."""
    idx, R, dR = nurbs3(patch, xi)
    P = patch.ctrl[..., :3].reshape(-1, 3)[idx]                  # [Q, L, 3]
    x = np.einsum("ql,qli->qi", R, P)
    J = np.einsum("qlj,qli->qij", dR, P)
    return x, J, idx, R, dR
