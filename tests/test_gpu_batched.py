"""Batched form: many independent scan strategies of uneven length on one
patch, advanced together by the HIP path, each checked against its own FP64
oracle run (or against a single-path HIP run where an oracle run per path
would be too slow)."""
import numpy as np
import pytest

from oracle import solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _model(patch, scan, **kw):
    from paper_2511_20432_amd import sa_iga
    return sa_iga.Model(patch, W.MAT_CFG, scan, kw.pop("options", None), **kw)


def _track(i, n_s=5, dt=1e-5):
    """Short straight track i on the small block: direction, power and speed vary with i."""
    rng = np.random.default_rng(100 + i)
    ang = rng.uniform(0, 2 * np.pi)
    c = np.array([0.5e-3, 0.3e-3, 0.5e-3])
    d = np.array([np.cos(ang), np.sin(ang) * 0.6, 0.0]) * 0.35e-3
    seg = W.Segment("line", float(rng.uniform(40, 120)), float(rng.uniform(0.6, 1.5)), p0=c - d, p1=c + d)
    return W.sources_from_segments([seg], dt / n_s)


def _check_path(gm, scan, p, n):
    om = solver.Model(W.small_block(), W.MAT_CFG, scan, path=p)
    om.advance(n)
    T, G, F, du = gm.boundary_fields(p)
    Tr, Gr = om.boundary_field(n)
    errs = {"T": rel(T, Tr), "grad": rel(G, Gr)}
    if np.abs(om.F).max() > 0:
        errs["F"] = rel(F, om.F)
        errs["du"] = rel(du, om.w)
    else:
        errs["F"] = float(np.abs(F).max())
        errs["du"] = float(np.abs(du).max())
    print(f"path {p} step {n}", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) <= TOL64, errs


def test_uneven_paths_match_oracle():
    """Five strategies, lengths 3..14 steps, one with no sources: paths drop
    out of the lockstep batch as they finish."""
    tracks = [_track(i) for i in range(4)]
    empty = (np.zeros((0, 3)), np.zeros(0, np.int64), np.zeros(0))
    scan = W.make_scan([tracks[0], tracks[1], empty, tracks[2], tracks[3]], 1e-5, 5,
                       n_steps=[3, 9, 5, 14, 12])
    gm = _model(W.small_block(), scan)
    gm.step(4)
    assert [gm.get_step(p) for p in range(5)] == [3, 4, 4, 4, 4]
    _check_path(gm, scan, 0, 3)
    gm.step(20)
    assert [gm.get_step(p) for p in range(5)] == [3, 9, 5, 14, 12]
    for p, n in ((1, 9), (2, 5), (3, 14), (4, 12)):
        _check_path(gm, scan, p, n)


def test_batched_equals_single_path_runs():
    """More paths than one launch holds (two lockstep groups), each path's
    result matches a separate one-path HIP run of the same strategy."""
    n_paths = 67
    tracks = [_track(i) for i in range(n_paths)]
    steps = [2 + (i % 3) for i in range(n_paths)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=steps)
    gm = _model(W.small_block(), scan)
    gm.step(5)
    st = gm.stats()
    assert st["steps"] == sum(steps)
    for p in (0, 1, 63, 64, 65, 66):
        one = _model(W.small_block(), scan.path(p))
        one.step(steps[p])
        for a, b, name in zip(gm.boundary_fields(p), one.boundary_fields(), ("T", "grad", "F", "du")):
            # the chunking of the source history depends on the batch size
            assert rel(a, b) <= 1e-12, (p, name, rel(a, b))
    _check_path(gm, scan, 65, steps[65])


def test_batched_fp32_far_within_005K():
    """FP32 far field with per-path far/near splits in one launch."""
    tracks = [_track(i) for i in range(3)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[40, 25, 33])
    opts = W.Options(precision=W.PRECISION_FP32_FAR, tau_near=5e-5)
    gm = _model(W.small_block(), scan, options=opts)
    gm.step(40)
    st = gm.stats()
    assert 0 < st["pairs_near"] < st["pairs"]
    for p, n in ((0, 40), (1, 25), (2, 33)):
        om = solver.Model(W.small_block(), W.MAT_CFG, scan, path=p)
        om.advance(n)
        R = om.bt["R"]
        T, G, F, du = gm.boundary_fields(p)
        Tr, Gr = om.boundary_field(n)
        err = np.abs((T + R @ du) - (Tr + R @ om.w)).max()
        print(f"fp32-far path {p}: max |T - T_ref| = {err:.3e} K", flush=True)
        assert err <= 0.05


def test_batched_checkpoint_resume_bitwise():
    tracks = [_track(i) for i in range(3)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[6, 11, 9])
    a = _model(W.small_block(), scan)
    b = _model(W.small_block(), scan)
    a.step(7)                       # path 0 has finished; the others are mid-scan
    blob = a.save()
    a.step(6)
    b.step(3)
    b.load(blob)
    b.step(6)
    for p in range(3):
        assert a.get_step(p) == b.get_step(p)
        for x, y in zip(a.boundary_fields(p), b.boundary_fields(p)):
            assert np.array_equal(x, y)


def test_paths_at_different_steps_share_launches():
    """A checkpoint with paths at steps 3, 5, 2, 5 continued under longer
    scans: paths at different steps (same parity) advance in one launch."""
    tracks = [_track(i) for i in range(4)]
    short = W.make_scan(tracks, 1e-5, 5, n_steps=[3, 5, 2, 8])
    a = _model(W.small_block(), short)
    a.step(5)
    assert [a.get_step(p) for p in range(4)] == [3, 5, 2, 5]
    long = W.make_scan(tracks, 1e-5, 5, n_steps=[10, 10, 10, 10])
    b = _model(W.small_block(), long)
    b.load(a.save())
    for p in range(4):
        for x, y in zip(a.boundary_fields(p), b.boundary_fields(p)):
            assert np.array_equal(x, y)
    b.step(4)
    assert [b.get_step(p) for p in range(4)] == [7, 9, 6, 9]
    for p, n in ((0, 7), (1, 9), (2, 6), (3, 9)):
        _check_path(b, long, p, n)


def test_tile_shapes_bitwise_equal_and_autotune(monkeypatch):
    """The pair-by-pair kernel's tile shape changes no bit of any result; the
    tuner picks a valid shape and leaves the state alone.  The block's faces
    are tensor faces, so the pair-by-pair kernel is forced on them here
    (SA_IGA_NO_TENSOR); with the matrix-core sum the tuner times one shape."""
    tracks = [_track(i) for i in range(3)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[12, 9, 12])
    tens = _model(W.small_block(), scan)
    assert tens.info.generic_points == 0
    t = tens.autotune(reps=2)
    assert (t["points_per_lane"], t["waves_per_group"]) == (2, 4) and t["ms_per_step"] > 0
    monkeypatch.setenv("SA_IGA_NO_TENSOR", "1")
    for prec in (W.PRECISION_FP64, W.PRECISION_FP32_FAR):
        opts = W.Options(precision=prec, tau_near=5e-5)
        a = _model(W.small_block(), scan, options=opts, points_per_lane=1, waves_per_group=1)
        b = _model(W.small_block(), scan, options=opts, points_per_lane=4, waves_per_group=8)
        assert b.info.generic_points == b.info.n_bpts
        a.step(6)
        b.step(6)
        before = [b.boundary_fields(p) for p in range(3)]
        t = b.autotune(reps=2)
        print("autotune", prec, t, flush=True)
        assert t["points_per_lane"] in (1, 2, 4) and t["waves_per_group"] in (1, 2, 4, 8)
        assert t["ms_per_step"] > 0
        for p in range(3):
            for x, y in zip(before[p], b.boundary_fields(p)):
                assert np.array_equal(x, y)
        a.step(6)
        b.step(6)
        for p in range(3):
            for x, y in zip(a.boundary_fields(p), b.boundary_fields(p)):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("n_paths", [1, 5])
def test_tensor_launch_shape_tuning_changes_no_bit(n_paths):
    """The tuner's choice of the matrix-core sum's launch shape (workgroups
    per compute unit and LDS padding with five paths; LDS padding and block length for the
    blocked one-path calls) is a valid one and changes no result bit."""
    tracks = [_track(i) for i in range(n_paths)]
    scan = W.make_scan(tracks, 1e-5, 5, n_steps=[60] * n_paths)
    opts = W.Options(precision=W.PRECISION_FP32_FAR, tau_near=5e-5)
    a = _model(W.cfg1().patch, scan, options=opts)
    b = _model(W.cfg1().patch, scan, options=opts)
    t = b.autotune(reps=2)
    print("tuned", n_paths, "paths:", t, flush=True)
    if n_paths >= 4:
        assert t["sum_groups_per_cu_batch"] in (4, 6, 8, 12) and t["batch_lds_pad"] in (0, 10000, 38000)
    else:
        assert t["block_lds_pad"] in (0, 10000, 38000) and t["blocked_steps"] in (4, 8)
    for k in (7, 30, 23):
        a.step(k)
        b.step(k)
        for p in range(n_paths):
            for x, y in zip(a.boundary_fields(p), b.boundary_fields(p)):
                assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", [W.PRECISION_FP64, W.PRECISION_FP32_FAR])
def test_overlapped_steps_equal_serial_bitwise(monkeypatch, prec):
    """The source side of step n+2 (sum, load vector, Dirichlet data) runs on
    a stream of its own beside the theta-step solve of step n+1.  The results
    are bitwise those of the serial order, here with 67 paths at mixed step
    parities (several launch groups), stage timing on and off, and a
    checkpoint taken between calls."""
    n = 67
    tracks = [_track(i) for i in range(n)]
    short = W.make_scan(tracks, 1e-5, 5, n_steps=[3 + i % 4 for i in range(n)])
    long = W.make_scan(tracks, 1e-5, 5, n_steps=[14] * n)
    opts = W.Options(precision=prec, tau_near=5e-5)
    seed = _model(W.small_block(), short, options=opts)
    seed.step(6)
    blob = seed.save()
    monkeypatch.setenv("SA_IGA_SERIAL", "1")
    ser = _model(W.small_block(), long, options=opts)
    monkeypatch.delenv("SA_IGA_SERIAL")
    ovl = _model(W.small_block(), long, options=opts)
    for m in (ser, ovl):
        m.load(blob)
    ovl.set_timing(True)
    for k in (1, 4):
        ser.step(k)
        ovl.step(k)
    mid = ovl.save()
    ovl.set_timing(False)
    for k in (5, 2):
        ser.step(k)
        ovl.step(k)
    st = ovl.stats()
    print(f"overlapped: {st['steps']} path-steps, stage ms {st['stage_ms']}", flush=True)
    for p in range(n):
        assert ser.get_step(p) == ovl.get_step(p)
        for x, y in zip(ser.boundary_fields(p), ovl.boundary_fields(p)):
            assert np.array_equal(x, y)
    # resuming from the checkpoint taken between overlapped calls
    ovl.load(mid)
    ovl.step(7)
    for p in range(n):
        for x, y in zip(ser.boundary_fields(p), ovl.boundary_fields(p)):
            assert np.array_equal(x, y)
