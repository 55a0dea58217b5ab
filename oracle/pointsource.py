"""Analytical field of the discretised laser (paper Sec. 2.1, Eqs. 7-8).

Test infrastructure only (see the package docstring).

One instantaneous point source I with energy E, located at x_I and switched
on at t_I, gives in the unbounded medium (Eq. 8)

    T~_I(x, t) = s E / (rho c_p [4 pi alpha D]^{3/2}) exp(-|x - x_I|^2 / (4 alpha D)),
    D = t - tau_I,  tau_I = t_I - r^2/(8 alpha)   (finite spot, text after Eq. 8)

with alpha = k/(rho c_p) (Eq. 2); the field T~ is the sum over the sources
switched on so far (Eq. 7).  Its gradient is
    grad T~_I = T~_I * (-(x - x_I) / (2 alpha D)).

Readings:
  * s is a kernel scale, 1 by default (Eq. 8 as printed);
  * causality is decided on integer ticks: with delta = dt / sources_per_step
    and t = step * dt, a source with tick k is active iff k*delta <= t, and
    t - t_I = (step*sources_per_step - k) * delta is formed from the integer
    age;
  * absorbed power is given, so E = P_abs * delta (the paper's E = A P dt
    with A already applied).
"""
from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np


def diffusivity(material):
    return material.k / (material.rho * material.cp)


def kernel(x, src_xyz, D, energy, material, s=1.0):
    """T~ and grad T~ of individual sources: x [Q,3], src_xyz [S,3], D [S]
    (seconds, t - tau_I > 0), energy [S].  Returns T [Q,S], G [Q,S,3]."""
    a = diffusivity(material)
    rc = material.rho * material.cp
    dx = x[:, None, :] - src_xyz[None, :, :]
    R2 = np.sum(dx * dx, axis=-1)
    amp = s * energy / (rc * (4.0 * np.pi * a * D) ** 1.5)
    T = amp[None, :] * np.exp(-R2 / (4.0 * a * D[None, :]))
    G = T[:, :, None] * (-dx / (2.0 * a * D[None, :, None]))
    return T, G


def _field_block(x, xs, D, E, material, s):
    """Sum of Eq. 8 over the sources for a block of points, one coordinate
    at a time (same arithmetic as kernel(), fewer temporaries)."""
    a = diffusivity(material)
    rc = material.rho * material.cp
    amp = s * E / (rc * (4.0 * np.pi * a * D) ** 1.5)
    d0 = x[:, 0, None] - xs[None, :, 0]
    d1 = x[:, 1, None] - xs[None, :, 1]
    d2 = x[:, 2, None] - xs[None, :, 2]
    R2 = d0 * d0 + d1 * d1 + d2 * d2
    T = amp[None, :] * np.exp(-R2 / (4.0 * a * D[None, :]))
    Tb = T * (-1.0 / (2.0 * a * D))[None, :]
    G = np.stack([np.einsum("qs,qs->q", Tb, d0), np.einsum("qs,qs->q", Tb, d1),
                  np.einsum("qs,qs->q", Tb, d2)], axis=1)
    return T.sum(axis=1), G


def field(x, src_xyz, tick, energy, step, scan, material, s=1.0, threads=None):
    """Superposition (Eq. 7) at time t = step * dt over the active sources.

    Returns T [Q] and grad [Q, 3].  Blocks of points are summed on a thread
    pool (numpy releases the GIL inside its loops)."""
    a = diffusivity(material)
    now = step * scan.sources_per_step
    act = tick <= now
    age = (now - tick[act]).astype(np.float64)
    D = age * scan.delta + scan.spot_radius ** 2 / (8.0 * a)
    xs, E = src_xyz[act], energy[act]
    T = np.zeros(len(x))
    G = np.zeros((len(x), 3))
    if len(D) == 0 or len(x) == 0:
        return T, G
    chunk = max(1, int(250_000 // len(D)))
    blocks = [(c0, min(c0 + chunk, len(x))) for c0 in range(0, len(x), chunk)]

    def run(b):
        T[b[0]:b[1]], G[b[0]:b[1]] = _field_block(x[b[0]:b[1]], xs, D, E, material, s)

    n_thr = threads if threads is not None else default_threads()
    if n_thr <= 1 or len(blocks) == 1:
        for b in blocks:
            run(b)
    else:
        with _cf.ThreadPoolExecutor(n_thr) as ex:
            list(ex.map(run, blocks))
    return T, G


def default_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))
