"""FP64 forward and backward of the far-history network, and its input features.

Test infrastructure only (see the package docstring).

The surrogate form replaces the far part of the superposition (Eq. 7 over
the sources older than tau_near) at a boundary point by a small network.
The paper has no such network; its definition here is the reading both
sides implement:

  features (70): [xn (3), n (3), s (64)]
    xn = 2 (x - lo) / (hi - lo) - 1 per axis, with [lo, hi] the bounding box
         of the patch's control net;
    n  = outward unit normal at the point;
    s  = energy of the far sources (tick < now - tau_ticks, tick <= now)
         binned on a 4 x 4 x 4 grid over the same box: bin index per axis
         floor(4 (x_I - lo) / (hi - lo)) clamped to 0..3, flat index
         i0 + 4 i1 + 16 i2, each bin divided by E_scale.
  network: z1 = W1 x + b1 (W1: 256 x 70), h1 = gelu(z1);
           z_l = W_l h_{l-1} + b_l, h_l = gelu(z_l) for l = 2, 3, 4 (256 x 256);
           y = W5 h4 + b5 (W5: 4 x 256);
           gelu(z) = z (1 + erf(z / sqrt 2)) / 2.
  outputs: T~_far = T_scale y0, grad T~_far = G_scale (y1, y2, y3).
  loss: mean over samples and the four outputs of (y - t)^2 with the
        targets t scaled the same way.

Precision of the GPU network, which `forward(..., bf16=True)` reproduces
at the same rounding points (so the comparison measures accumulation order
and the GPU's GELU, the tanh form of Hendrycks & Gimpel, within 4.7e-4 of
the erf form defined here):
the hidden products W_l h_{l-1} (l = 2..4) take both operands rounded to
bfloat16 and accumulate in FP32; the activations h1..h4 are stored in
bfloat16; the first and the output layer use FP32 weights.  In the backward
pass the products with W_l (l = 2..4) and for their weight gradients take
dz_l rounded to bfloat16.  With bf16=False everything is FP64, which is what
the finite-difference pins check.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN = 70
N_HID = 256
N_OUT = 4
N_BINS = 64

LAYERS = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)),
          ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)),
          ("W4", (N_HID, N_HID)), ("b4", (N_HID,)),
          ("W5", (N_OUT, N_HID)), ("b5", (N_OUT,)))


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), via FP32, returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def box_of(ctrl_xyzw):
    """Bounding box [lo, hi] of a control net [..., 4]."""
    p = np.asarray(ctrl_xyzw, dtype=np.float64).reshape(-1, 4)[:, :3]
    return p.min(axis=0), p.max(axis=0)


def point_features(x, n, lo, hi):
    """[Q, 6]: box-normalised position and the normal."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    n = np.asarray(n, dtype=np.float64).reshape(-1, 3)
    xn = 2.0 * (x - lo) / (hi - lo) - 1.0
    return np.concatenate([xn, n], axis=1)


def far_bins(xyz, tick, energy, now, tau_ticks, lo, hi, e_scale):
    """Far-history energy per bin (64), in units of e_scale."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    tick = np.asarray(tick)
    s = np.zeros(N_BINS)
    for i in range(len(tick)):
        if not (tick[i] <= now and tick[i] < now - tau_ticks):
            continue
        idx = [min(3, max(0, int(np.floor(4.0 * (xyz[i, d] - lo[d]) / (hi[d] - lo[d]))))) for d in range(3)]
        s[idx[0] + 4 * idx[1] + 16 * idx[2]] += energy[i]
    return s / e_scale


def features(x, n, bins, lo, hi):
    """[Q, 70] network inputs for points x, n with one far-energy summary."""
    pf = point_features(x, n, lo, hi)
    return np.concatenate([pf, np.broadcast_to(np.asarray(bins, float), (len(pf), N_BINS))], axis=1)


def forward(params, X, bf16=True):
    """y [B, 4] and the cache for backward.  X [B, 70]."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    if bf16:
        X = np.asarray(X, dtype=np.float32).astype(np.float64)
    z = [None] * 5
    h = [None] * 5
    z[1] = X @ params["W1"].T + params["b1"]
    h[1] = r(gelu(z[1]))
    for l in (2, 3, 4):
        z[l] = h[l - 1] @ r(params[f"W{l}"]).T + params[f"b{l}"]
        h[l] = r(gelu(z[l]))
    y = h[4] @ params["W5"].T + params["b5"]
    return y, {"X": X, "z": z, "h": h}


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t, bf16=True):
    """Gradients of mse(y, t) w.r.t. every parameter and the input."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    z, h, X = cache["z"], cache["h"], cache["X"]
    B = y.shape[0]
    g = {}
    dy = 2.0 * (y - t) / (B * N_OUT)
    g["W5"] = dy.T @ h[4]
    g["b5"] = dy.sum(axis=0)
    dh = dy @ params["W5"]
    for l in (4, 3, 2):
        dz = r(dh * gelu_grad(z[l]))
        g[f"W{l}"] = dz.T @ h[l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        dh = dz @ r(params[f"W{l}"])
    dz1 = dh * gelu_grad(z[1])
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    g["X"] = dz1 @ params["W1"]
    return g


def flatten(params):
    """FP32 parameter vector in the order of LAYERS (the weight blob body)."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).reshape(-1) for k, _ in LAYERS])


def unflatten(vec):
    vec = np.asarray(vec, dtype=np.float64)
    out, o = {}, 0
    for k, shp in LAYERS:
        n = int(np.prod(shp))
        out[k] = vec[o:o + n].reshape(shp)
        o += n
    if o != len(vec):
        raise ValueError(f"parameter vector has {len(vec)} values, the network {o}")
    return out


def n_params():
    return sum(int(np.prod(s)) for _, s in LAYERS)
