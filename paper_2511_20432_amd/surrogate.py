"""Far-history network: initial weights, training set from the exact far
sums of the library, training with the library's GPU kernels, and the weight
vector the surrogate form takes (sa_solver_options.surrogate_weights).

Marshalling and bookkeeping only: the far sums, the network's forward and
backward passes and the Adam updates run in libsa_iga's HIP kernels; torch
holds the device arrays.
"""
from __future__ import annotations

import time
from typing import List, Optional, Sequence

import numpy as np

from . import sa_iga
from . import workloads as W

N_IN, N_HID, N_OUT = 70, 256, 4
SHAPES = (("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)), ("W4", (N_HID, N_HID)), ("b4", (N_HID,)),
          ("W5", (N_OUT, N_HID)), ("b5", (N_OUT,)))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, a small output layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for name, shp in SHAPES:
        if name.startswith("b"):
            out.append(np.zeros(shp))
        elif name == "W5":
            out.append(rng.normal(size=shp) * 0.1 * np.sqrt(1.0 / shp[1]))
        else:
            out.append(rng.normal(size=shp) * np.sqrt(2.0 / shp[1]))
    return np.concatenate([a.reshape(-1) for a in out]).astype(np.float32)


def weights_blob(params: np.ndarray, t_scale: float, g_scale: float, e_scale: float) -> np.ndarray:
    return np.concatenate([np.array([t_scale, g_scale, e_scale], np.float32),
                           np.asarray(params, np.float32)])


def strategy_scan(seeds: Sequence[int], n_s: int = 5, dt: float = 1e-5) -> W.ScanPath:
    """One scan strategy per seed on the raster block (the batched workload's rules)."""
    paths, steps = [], []
    for sd in seeds:
        rng = np.random.Generator(np.random.PCG64(sd))
        segs, L, _, _, _ = W.strategy_segments(rng)
        paths.append(W.sources_from_segments(segs, dt / n_s, max_sources=L * n_s))
        steps.append(L)
    return W.make_scan(paths, dt, n_s, n_steps=steps)


def training_set(patch: W.Patch, scan: W.ScanPath, n_samples: int, e_scale: float, seed: int = 0,
                 points_per_draw: int = 4096, tau_near: float = 2e-4):
    """(X [n, 70] float32, T [n] float64, G [n, 3] float64) device tensors:
    the network inputs and the exact far field at random boundary points of
    random (strategy, step) pairs."""
    import torch
    m = sa_iga.Model(patch, W.MAT_CFG, scan, W.Options(tau_near=tau_near))
    rng = np.random.Generator(np.random.PCG64(seed))
    nq = m.info.n_bpts
    draws = int(np.ceil(n_samples / points_per_draw))
    Xs, Ts, Gs = [], [], []
    for _ in range(draws):
        p = int(rng.integers(scan.n_paths))
        L = int(scan.n_steps[p])
        step = int(rng.integers(1, L + 1))
        X, T, G = m.far_field(step, e_scale, path=p)
        idx = torch.from_numpy(rng.choice(nq, size=min(points_per_draw, nq), replace=False)).cuda()
        Xs.append(X[idx])
        Ts.append(T[idx])
        Gs.append(G[:, idx].T)
    X = torch.cat(Xs)[:n_samples].contiguous()
    T = torch.cat(Ts)[:n_samples].contiguous()
    G = torch.cat(Gs)[:n_samples].contiguous()
    m.close()
    return X, T, G


def scales_of(T, G):
    """Output scales: the 99.9th percentile of |T~_far| and of |grad T~_far|."""
    import torch
    t = float(torch.quantile(T.abs().float()[:1_000_000], 0.999))
    g = float(torch.quantile(G.abs().float().reshape(-1)[:1_000_000], 0.999))
    return max(t, 1e-6), max(g, 1e-6)


def targets(T, G, t_scale: float, g_scale: float):
    import torch
    return torch.cat([(T / t_scale)[:, None], G / g_scale], dim=1).float().contiguous()


def train(net: sa_iga.Mlp, X, Y, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          lr_final: Optional[float] = None, log=None) -> List[float]:
    """Adam over shuffled minibatches; cosine decay from lr to lr_final. Returns the mean loss per epoch."""
    import torch
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    lr_final = lr * 0.05 if lr_final is None else lr_final
    n_b = max(1, n // batch)
    total = epochs * n_b
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).cuda()
        acc = 0.0
        t0 = time.perf_counter()
        for b in range(n_b):
            idx = perm[b * batch:(b + 1) * batch]
            xb = X[idx].contiguous()
            yb = Y[idx].contiguous()
            a = lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * k / max(1, total - 1)))
            acc += net.train_step(xb, yb, float(a))
            k += 1
        hist.append(acc / n_b)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return hist
