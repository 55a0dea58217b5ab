"""Closed-form solutions used as pins (not part of the oracle).

  * Rosenthal's quasi-steady solution for a point source moving at constant
    speed in an unbounded medium: T - T0 = P/(4 pi k R) exp(-v (xi + R) / (2 alpha)),
    xi the coordinate along the motion relative to the source.
  * Mass of the Gaussian instantaneous source inside an axis-aligned box:
    a product of erf differences per axis.
  * Image lattice of a rectangular block (method of images): even images
    across adiabatic planes, odd images across the Dirichlet plane z = 0.
"""
import math

import numpy as np
from scipy.special import erf


def rosenthal(P, v, k, alpha, xi, R):
    return P / (4.0 * math.pi * k * R) * np.exp(-v * (xi + R) / (2.0 * alpha))


def gaussian_box_fraction(src, D, alpha, lo, hi):
    """Fraction of the instantaneous source's energy inside the box [lo, hi]
    after time-like parameter D (variance 2 alpha D per axis)."""
    s = math.sqrt(4.0 * alpha * D)
    f = 1.0
    for d in range(3):
        f *= 0.5 * (erf((hi[d] - src[d]) / s) - erf((lo[d] - src[d]) / s))
    return f


def image_lattice(src, size, n_img=3):
    """Images of a source at src in the box [0, Lx] x [0, Ly] x [0, H] with
    adiabatic x, y planes and top, Dirichlet bottom (z = 0), source on the
    top plane (src z = H).  Returns list of (position, sign), the identity
    image first."""
    Lx, Ly, H = size
    xs = []
    for j in range(-n_img, n_img + 1):
        xs.append(src[0] + 2 * j * Lx)
        xs.append(-src[0] + 2 * j * Lx)
    ys = []
    for j in range(-n_img, n_img + 1):
        ys.append(src[1] + 2 * j * Ly)
        ys.append(-src[1] + 2 * j * Ly)
    assert abs(src[2] - H) < 1e-15
    zs = []
    for m in range(0, n_img + 1):
        zs.append(((2 * m + 1) * H, (-1) ** m))
        zs.append((-(2 * m + 1) * H, -((-1) ** m)))
    out = []
    ident = (src[0], src[1], H)
    for x in xs:
        for y in ys:
            for z, sg in zs:
                out.append(((x, y, z), sg))
    # identity image first; coinciding positions (a source on a lateral
    # plane) are kept: the pair doubles the field as the half-space requires
    out.sort(key=lambda e: 0 if np.allclose(e[0], ident, atol=1e-18) and e[1] > 0 else 1)
    return out
