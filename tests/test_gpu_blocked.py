"""Blocked source side: a call of one path (or a few at one step parity)
computes the kernel sums, reductions, load vectors and Dirichlet data of up
to eight steps per launch, then runs the theta-steps of the block.  The
results are bitwise those of the one-step serial order, for call lengths
that end blocks early, with a checkpoint taken between calls, and for two
paths per block."""
import numpy as np
import pytest

from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu


def _model(patch, scan, **kw):
    from paper_2511_20432_amd import sa_iga
    return sa_iga.Model(patch, W.MAT_CFG, scan, kw.pop("options", None), **kw)


def _track(i, n_s=5, dt=1e-5):
    rng = np.random.default_rng(300 + i)
    ang = rng.uniform(0, 2 * np.pi)
    c = np.array([0.5e-3, 0.3e-3, 0.5e-3])
    d = np.array([np.cos(ang), np.sin(ang) * 0.6, 0.0]) * 0.35e-3
    seg = W.Segment("line", float(rng.uniform(40, 120)), float(rng.uniform(0.6, 1.5)), p0=c - d, p1=c + d)
    return W.sources_from_segments([seg], dt / n_s)


def _pair(monkeypatch, scan, opts):
    monkeypatch.setenv("SA_IGA_SERIAL", "1")
    ser = _model(W.small_block(), scan, options=opts)
    monkeypatch.delenv("SA_IGA_SERIAL")
    blk = _model(W.small_block(), scan, options=opts)
    assert ser.info.blocked_steps == 1 and blk.info.blocked_steps == 8
    assert blk.info.n_dirichlet > 0
    return ser, blk


def _equal(a, b, paths):
    for p in paths:
        assert a.get_step(p) == b.get_step(p)
        for x, y in zip(a.boundary_fields(p), b.boundary_fields(p)):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", [W.PRECISION_FP64, W.PRECISION_FP32_FAR])
def test_blocked_one_path_equals_serial_bitwise(monkeypatch, prec):
    scan = W.make_scan([_track(0)], 1e-5, 5, n_steps=[41])
    opts = W.Options(precision=prec, tau_near=5e-5)
    ser, blk = _pair(monkeypatch, scan, opts)
    for k in (5, 1, 11):            # blocks of 5; 1; 8 + 3
        ser.step(k)
        blk.step(k)
        _equal(ser, blk, [0])
    mid = blk.save()
    ser.step(30)                    # runs past the end of the scan
    blk.step(30)
    _equal(ser, blk, [0])
    st = blk.stats()
    print(f"blocked: {st['steps']} steps, rollbacks {st['rollbacks']}, PCG iterations {st['pcg_iterations']}",
          flush=True)
    assert st["rollbacks"] == 0 and st["pcg_iterations"] == st["steps"] == 41
    blk.load(mid)
    blk.step(25)
    _equal(ser, blk, [0])


def test_blocked_two_paths_equal_serial_bitwise(monkeypatch):
    """Two paths of different lengths: blocks of four steps of both, then
    of eight steps of the longer one once the shorter has finished."""
    scan = W.make_scan([_track(1), _track(2)], 1e-5, 5, n_steps=[13, 30])
    ser, blk = _pair(monkeypatch, scan, W.Options())
    ser.step(30)
    blk.step(30)
    _equal(ser, blk, [0, 1])


def test_blocked_without_dirichlet_faces(monkeypatch):
    """No Dirichlet face (the bottom face Neumann as well): the blocked
    schedule without Dirichlet data matches the serial order bitwise and the
    oracle to 1e-9."""
    from oracle import solver
    roles = (W.FACE_NEUMANN,) * 5 + (W.FACE_SOURCE_PLANE,)
    patch = W.small_block(roles=roles)
    scan = W.make_scan([_track(3)], 1e-5, 5, n_steps=[19])
    monkeypatch.setenv("SA_IGA_SERIAL", "1")
    ser = _model(patch, scan)
    monkeypatch.delenv("SA_IGA_SERIAL")
    blk = _model(patch, scan)
    assert blk.info.n_dirichlet == 0 and blk.info.blocked_steps == 8
    for k in (7, 12):
        ser.step(k)
        blk.step(k)
    _equal(ser, blk, [0])
    om = solver.Model(patch, W.MAT_CFG, scan)
    om.advance(19)
    T, G, F, du = blk.boundary_fields()
    Tr, Gr = om.boundary_field(19)
    for a, b in ((T, Tr), (G, Gr), (F, om.F), (du, om.w)):
        b = np.asarray(b)
        err = float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))
        assert err <= 1e-9, err
