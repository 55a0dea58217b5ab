"""Pins of the oracle's far-history network and features (oracle/mlp.py):
closed forms of GELU, bfloat16 rounding against a library conversion and
hand-worked bit patterns, hand-binned far energy, a network whose output is
known in closed form, and the backward pass against central finite
differences."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {}
    for k, shp in mlp.LAYERS:
        fan_in = shp[1] if len(shp) == 2 else 1
        p[k] = rng.normal(size=shp) * (scale * np.sqrt(2.0 / fan_in) if len(shp) == 2 else 0.1)
    return p


def test_gelu_closed_forms():
    z = np.linspace(-6, 6, 101)
    # erf is odd: gelu(z) - gelu(-z) = z
    assert np.abs(mlp.gelu(z) - mlp.gelu(-z) - z).max() < 1e-15
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-16
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-15 and abs(mlp.gelu(-10.0)) < 1e-20
    # gelu(1) = Phi(1) with Phi the standard normal CDF: 0.8413447460685429
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-9


def test_bf16_round_bit_patterns_and_library():
    one = 1.0
    assert mlp.bf16_round(one) == 1.0
    assert mlp.bf16_round(1 + 2.0 ** -8) == 1.0                   # tie -> even mantissa
    assert mlp.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6      # tie -> even mantissa
    assert mlp.bf16_round(1 + 2.0 ** -8 + 2.0 ** -12) == 1 + 2.0 ** -7
    assert mlp.bf16_round(-3.0) == -3.0
    x = np.random.default_rng(1).normal(size=20000) * np.exp(np.random.default_rng(2).uniform(-20, 20, 20000))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_far_bins_by_hand():
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([4e-3, 2e-3, 1e-3])
    xyz = np.array([[0.1e-3, 0.1e-3, 1e-3],     # bin (0, 0, 3) -> 48
                    [3.9e-3, 1.9e-3, 1e-3],     # bin (3, 3, 3) -> 63
                    [2.0e-3, 1.0e-3, 0.5e-3],   # bin (2, 2, 2) -> 42
                    [2.0e-3, 1.0e-3, 0.5e-3],   # too young
                    [-1e-3, 5e-3, 1e-3]])       # clamped to (0, 3, 3) -> 60
    tick = np.array([1, 2, 3, 90, 4])
    E = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    s = mlp.far_bins(xyz, tick, E, now=100, tau_ticks=10, lo=lo, hi=hi, e_scale=2.0)
    want = np.zeros(64)
    want[48], want[63], want[42], want[60] = 0.5, 1.0, 2.0, 8.0
    assert np.array_equal(s, want)
    # the age bound is strict: tick = now - tau is near
    s2 = mlp.far_bins(xyz[:1], np.array([90]), E[:1], now=100, tau_ticks=10, lo=lo, hi=hi, e_scale=1.0)
    assert s2.sum() == 0.0
    # not yet switched on
    s3 = mlp.far_bins(xyz[:1], np.array([101]), E[:1], now=100, tau_ticks=-5, lo=lo, hi=hi, e_scale=1.0)
    assert s3.sum() == 0.0


def test_point_features():
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([4.0, 2.0, 1.0])
    f = mlp.point_features([[0, 0, 0], [4, 2, 1], [2, 1, 0.5]], [[1, 0, 0]] * 3, lo, hi)
    assert np.array_equal(f[:, :3], [[-1, -1, -1], [1, 1, 1], [0, 0, 0]])
    assert np.array_equal(f[:, 3:], [[1, 0, 0]] * 3)


def test_network_with_zero_weights_is_closed_form():
    p = _params(3)
    for l in (1, 2, 3, 4):
        p[f"W{l}"] = np.zeros_like(p[f"W{l}"])
    X = np.random.default_rng(4).normal(size=(5, mlp.N_IN))
    y, _ = mlp.forward(p, X, bf16=False)
    want = p["W5"] @ mlp.gelu(p["b4"]) + p["b5"]
    assert np.abs(y - want[None, :]).max() < 1e-13


def test_flatten_roundtrip_and_size():
    p = _params(5)
    v = mlp.flatten(p)
    assert len(v) == mlp.n_params() == 256 * 70 + 256 + 3 * (256 * 256 + 256) + 4 * 256 + 4
    q = mlp.unflatten(v)
    for k, _ in mlp.LAYERS:
        assert np.array_equal(p[k], q[k])
    with pytest.raises(ValueError):
        mlp.unflatten(v[:-1])


def test_backward_matches_central_differences():
    p = _params(6)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(6, mlp.N_IN))
    t = rng.normal(size=(6, mlp.N_OUT))
    y, cache = mlp.forward(p, X, bf16=False)
    g = mlp.backward(p, cache, y, t, bf16=False)

    def loss(pp, XX):
        return mlp.mse(mlp.forward(pp, XX, bf16=False)[0], t)

    h = 1e-6
    for k, shp in mlp.LAYERS:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k].reshape(-1)[idx] += h
            lp = loss(pp, X)
            pp[k].reshape(-1)[idx] -= 2 * h
            lm = loss(pp, X)
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (k, idx, fd, an)
    for b, j in ((0, 0), (3, 17), (5, 69)):
        Xp = X.copy()
        Xp[b, j] += h
        lp = loss(p, Xp)
        Xp[b, j] -= 2 * h
        lm = loss(p, Xp)
        assert abs((lp - lm) / (2 * h) - g["X"][b, j]) < 1e-8


def test_bf16_network_close_to_fp64():
    """The bfloat16 reading changes the output by about the bfloat16 epsilon."""
    p = _params(8)
    X = np.random.default_rng(9).normal(size=(64, mlp.N_IN))
    y64, _ = mlp.forward(p, X, bf16=False)
    y16, _ = mlp.forward(p, X, bf16=True)
    e = np.abs(y16 - y64).max() / np.abs(y64).max()
    assert 1e-5 < e < 5e-2
