"""The far-history network on the GPU (matrix-core forward, backward and
Adam through the C ABI) against the FP64 oracle of the same network, the
library's far-field training data against the oracle's kernel sum, and the
surrogate form of the step: network far field, audits and exact fallback."""
import numpy as np
import pytest
import torch

from oracle import iga, mlp, pointsource, solver
from paper_2511_20432_amd import surrogate
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _net(seed=0, bias=0.1):
    from paper_2511_20432_amd import sa_iga
    p = surrogate.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    # nonzero biases so that every term of the backward pass is exercised
    q = mlp.unflatten(p.astype(np.float64))
    for k in ("b1", "b2", "b3", "b4", "b5"):
        q[k] = rng.normal(size=q[k].shape) * bias
    p = mlp.flatten(q).astype(np.float32)
    return sa_iga.Mlp(p), p


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 70)).astype(np.float32)
    T = rng.normal(size=(B, 4)).astype(np.float32)
    return X, T


def test_forward_matches_oracle_ragged_batches():
    net, p = _net(0)
    P = mlp.unflatten(p.astype(np.float64))
    for B in (1, 37, 300, 1029):
        X, _ = _inputs(B, B)
        Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
        Yr, _ = mlp.forward(P, X, bf16=True)
        e = rel(Y, Yr)
        print(f"forward B={B}: rel {e:.2e}", flush=True)
        assert e <= 1e-2


def test_gradients_match_oracle():
    net, p = _net(2)
    P = mlp.unflatten(p.astype(np.float64))
    X, T = _inputs(515, 3)
    g, loss = net.gradients(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    y, cache = mlp.forward(P, X, bf16=True)
    gr = mlp.backward(P, cache, y, T.astype(np.float64), bf16=True)
    assert abs(loss - mlp.mse(y, T)) <= 1e-2 * mlp.mse(y, T)
    G = mlp.unflatten(g.astype(np.float64))
    for k, _ in mlp.LAYERS:
        e = rel(G[k], gr[k])
        print(f"grad {k}: rel {e:.2e}", flush=True)
        assert e <= 1e-2, k


def test_adam_step_and_training_reduce_loss():
    net, p = _net(4)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(4096, 70)).astype(np.float32)
    # a smooth target the network can fit
    T = np.stack([np.tanh(X[:, 0] + 0.5 * X[:, 6]), np.sin(X[:, 1]), X[:, 2] * X[:, 3] * 0.3,
                  0.2 * X[:, 7]], axis=1).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    # one Adam step moves every weight by about lr (bias-corrected first step)
    before = net.params()
    l0 = net.train_step(Xd, Td, 1e-3)
    after = net.params()
    d = np.abs(after - before)
    g, _ = net.gradients(Xd, Td)
    moved = d[np.abs(g) > 1e-6]
    assert np.median(moved) == pytest.approx(1e-3, rel=0.05)
    losses = [net.train_step(Xd, Td, 1e-3) for _ in range(300)]
    print(f"loss {l0:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.2 * l0


def test_far_field_and_inputs_match_oracle():
    from paper_2511_20432_amd import sa_iga
    patch = W.small_block()
    tr = surrogate_track()
    scan = W.make_scan([tr], 1e-5, 5, n_steps=[40])
    tau = 5e-5
    m = sa_iga.Model(patch, W.MAT_CFG, scan, W.Options(tau_near=tau))
    bt = iga.boundary_tables(patch)
    lo, hi = mlp.box_of(patch.ctrl)
    tau_ticks = int(np.floor(tau / (scan.dt / scan.sources_per_step) + 1e-9))
    for step in (3, 17, 40):
        X, T, G = m.far_field(step, 1e-3)
        now = step * scan.sources_per_step
        far = scan.tick < now - tau_ticks
        Tr, Gr = pointsource.field(bt["x"], scan.xyz[far], scan.tick[far], scan.energy[far], step, scan, W.MAT_CFG)
        if far.sum() == 0:
            assert T.abs().max().item() == 0.0
        else:
            assert rel(T.cpu().numpy(), Tr) <= 1e-9
            assert rel(G.cpu().numpy().T, Gr) <= 1e-9
        bins = mlp.far_bins(scan.xyz, scan.tick, scan.energy, now, tau_ticks, lo, hi, 1e-3)
        Xr = mlp.features(bt["x"], bt["n"], bins, lo, hi).astype(np.float32)
        Xg = X.cpu().numpy()
        assert np.abs(Xg[:, :6] - Xr[:, :6]).max() <= 1e-6
        assert np.abs(Xg[:, 6:] - Xr[:, 6:]).max() <= 1e-6 * max(1.0, np.abs(Xr[:, 6:]).max())


def surrogate_track():
    seg = W.Segment("line", 80.0, 1.0, p0=np.array([0.1e-3, 0.3e-3, 0.5e-3]), p1=np.array([0.9e-3, 0.3e-3, 0.5e-3]))
    return W.sources_from_segments([seg], 2e-6)


def _surrogate_model(scan, params, tau, t_scale=50.0, **kw):
    from paper_2511_20432_amd import sa_iga
    blob = surrogate.weights_blob(params, t_scale, 2e5, 1e-3)
    return sa_iga.Model(W.small_block(), W.MAT_CFG, scan, W.Options(precision=W.PRECISION_SURROGATE, tau_near=tau),
                        surrogate_weights=blob, **kw)


def test_surrogate_step_uses_network_far_field():
    """With an audit that always passes, T~ at the boundary points is the
    exact FP64 near sum plus T_scale times the network's first output."""
    tr = surrogate_track()
    scan = W.make_scan([tr], 1e-5, 5, n_steps=[30])
    tau = 5e-5
    _, p = _net(6)
    gm = _surrogate_model(scan, p, tau, audit_tol=1e30, audit_every=7)
    gm.step(30)
    st = gm.stats()
    # far sources from step 6 on (tick < 5 step - 25): audits at steps 6, 13,
    # 20 and 27, the network from the first passing one
    assert st["net_steps"] == 25 and st["audits"] == 4 and st["audit_failures"] == 0
    assert st["pairs_net"] > 0
    T, G, F, du = gm.boundary_fields()
    patch = W.small_block()
    bt = iga.boundary_tables(patch)
    lo, hi = mlp.box_of(patch.ctrl)
    now = 30 * scan.sources_per_step
    tau_ticks = int(np.floor(tau / (scan.dt / scan.sources_per_step) + 1e-9))
    near = (scan.tick <= now) & (scan.tick >= now - tau_ticks)
    Tn, Gn = pointsource.field(bt["x"], scan.xyz[near], scan.tick[near], scan.energy[near], 30, scan, W.MAT_CFG)
    bins = mlp.far_bins(scan.xyz, scan.tick, scan.energy, now, tau_ticks, lo, hi, 1e-3)
    X = mlp.features(bt["x"], bt["n"], bins, lo, hi)
    y, _ = mlp.forward(mlp.unflatten(p.astype(np.float64)), X, bf16=True)
    e_T = rel(T - Tn, 50.0 * y[:, 0])
    e_G = rel(G - Gn, 2e5 * y[:, 1:])
    print(f"network far field: T rel {e_T:.2e}, grad rel {e_G:.2e}", flush=True)
    assert e_T <= 1e-2 and e_G <= 1e-2


def test_surrogate_audit_falls_back_to_exact():
    """An untrained network fails every audit, so no step uses it: the path
    sums its far sources as the FP32 far-field form does, bitwise."""
    from paper_2511_20432_amd import sa_iga
    tr = surrogate_track()
    scan = W.make_scan([tr], 1e-5, 5, n_steps=[24])
    tau = 5e-5
    _, p = _net(7)
    gm = _surrogate_model(scan, p, tau, t_scale=1e4, audit_every=1)   # off by ~1000 K
    ref = sa_iga.Model(W.small_block(), W.MAT_CFG, scan, W.Options(precision=W.PRECISION_FP32_FAR, tau_near=tau))
    gm.step(24)
    ref.step(24)
    st = gm.stats()
    print("surrogate stats", {k: st[k] for k in ("net_steps", "audits", "audit_failures", "audit_max_err")},
          flush=True)
    # far sources from step 6 on: one audit per step from there
    assert st["audits"] == 19 and st["audit_failures"] == 19 and st["net_steps"] == 0
    for a, b in zip(gm.boundary_fields(), ref.boundary_fields()):
        assert np.array_equal(a, b)


def test_surrogate_never_runs_unaudited():
    """With the default audit period (50 steps) an untrained network is
    audited on the path's first step with far sources, before it is used:
    it fails, and every step equals the FP32 far-field form's bitwise."""
    from paper_2511_20432_amd import sa_iga
    tr = surrogate_track()
    scan = W.make_scan([tr], 1e-5, 5, n_steps=[40])
    tau = 5e-5
    _, p = _net(8)
    gm = _surrogate_model(scan, p, tau, t_scale=1e4)
    ref = sa_iga.Model(W.small_block(), W.MAT_CFG, scan, W.Options(precision=W.PRECISION_FP32_FAR, tau_near=tau))
    for k in (3, 4, 33):
        gm.step(k)
        ref.step(k)
        for a, b in zip(gm.boundary_fields(), ref.boundary_fields()):
            assert np.array_equal(a, b)
    st = gm.stats()
    assert st["audits"] == 1 and st["audit_failures"] == 1 and st["net_steps"] == 0


def test_surrogate_checkpoint_keeps_audit_state():
    """A checkpoint holds each path's audit state (network or exact far sum,
    step of the next audit): a run resumed from it in another object, whose
    own state differs, continues bitwise as the uninterrupted run, with the
    same audits.  Far sources start at step 6, so with audits every 5 steps
    the uninterrupted run audits at 6, 11, 16, 21; a resumed run that lost
    the state would audit at 13, 18, 23 instead."""
    tracks = [surrogate_track(), W.sources_from_segments(
        [W.Segment("line", 60.0, 0.8, p0=np.array([0.2e-3, 0.1e-3, 0.5e-3]),
                   p1=np.array([0.8e-3, 0.5e-3, 0.5e-3]))], 2e-6)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[30, 22])
    tau = 5e-5
    _, p = _net(11)
    a = _surrogate_model(scan, p, tau, audit_every=5, audit_tol=40.0)
    a.step(12)
    ck = a.save()
    s0 = a.stats()
    a.step(12)
    b = _surrogate_model(scan, p, tau, audit_every=5, audit_tol=40.0)
    b.step(2)                      # an unaudited state in memory
    b.load(ck)
    t0 = b.stats()
    b.step(12)
    s1, t1 = a.stats(), b.stats()
    d_a = {k: s1[k] - s0[k] for k in ("audits", "audit_failures", "net_steps", "pairs", "pairs_net")}
    d_b = {k: t1[k] - t0[k] for k in d_a}
    print("after the checkpoint", d_a, d_b, "; before", {k: s0[k] for k in ("audits", "audit_failures", "net_steps")},
          flush=True)
    assert d_a == d_b
    assert d_a["audits"] == 4
    for path in range(2):
        for x, y in zip(a.boundary_fields(path), b.boundary_fields(path)):
            assert np.array_equal(x, y)


def test_fused_network_matches_layerwise(monkeypatch):
    """The register-resident fused network and the layer-by-layer GEMM path
    give the same far field (to bfloat16 rounding of the activations)."""
    tr = surrogate_track()
    scan = W.make_scan([tr], 1e-5, 5, n_steps=[20])
    tau = 5e-5
    _, p = _net(9)
    a = _surrogate_model(scan, p, tau, audit_tol=1e30, audit_every=100)
    monkeypatch.setenv("SA_IGA_NET_LAYERWISE", "1")
    b = _surrogate_model(scan, p, tau, audit_tol=1e30, audit_every=100)
    a.step(20)
    b.step(20)
    Ta, Ga = a.boundary_fields()[:2]
    Tb, Gb = b.boundary_fields()[:2]
    e_T, e_G = rel(Ta, Tb), rel(Ga, Gb)
    print(f"fused vs layer-wise: T rel {e_T:.2e}, grad rel {e_G:.2e}", flush=True)
    assert e_T <= 1e-2 and e_G <= 1e-2


def test_surrogate_overlapped_equals_serial(monkeypatch):
    """The surrogate form (network far field, audits with host decisions)
    through the overlapped step pipeline gives bitwise the serial order's
    results, with audits that fail on some steps and pass on others."""
    tracks = [surrogate_track(), W.sources_from_segments(
        [W.Segment("line", 60.0, 0.8, p0=np.array([0.2e-3, 0.1e-3, 0.5e-3]),
                   p1=np.array([0.8e-3, 0.5e-3, 0.5e-3]))], 2e-6)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[26, 19])
    tau = 5e-5
    _, p = _net(11)
    monkeypatch.setenv("SA_IGA_SERIAL", "1")
    ser = _surrogate_model(scan, p, tau, audit_every=4, audit_tol=40.0)
    monkeypatch.delenv("SA_IGA_SERIAL")
    ovl = _surrogate_model(scan, p, tau, audit_every=4, audit_tol=40.0)
    for k in (3, 9, 14):
        ser.step(k)
        ovl.step(k)
    a, b = ser.stats(), ovl.stats()
    print("surrogate stats", {k: (a[k], b[k]) for k in ("net_steps", "audits", "audit_failures")}, flush=True)
    for k in ("net_steps", "audits", "audit_failures", "pairs", "pairs_net"):
        assert a[k] == b[k]
    for path in range(2):
        for x, y in zip(ser.boundary_fields(path), ovl.boundary_fields(path)):
            assert np.array_equal(x, y)
