"""The kernel sum on tensor faces (matrix products on the matrix cores)
against the pair-by-pair kernel of the same library (SA_IGA_NO_TENSOR at
set-up selects it), and the detection of the faces: every face of an
axis-aligned block, only the two planar end faces of the quarter annulus.
Both paths are checked against the oracle elsewhere; here they are checked
against each other on ragged tiles (face grids of 12 x 9 and 48 x 24 points)
and with several paths in one launch."""
import numpy as np
import pytest

from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _tracks(n):
    out = []
    for i in range(n):
        rng = np.random.default_rng(300 + i)
        ang = rng.uniform(0, 2 * np.pi)
        c = np.array([0.5e-3, 0.3e-3, 0.5e-3])
        d = np.array([np.cos(ang), np.sin(ang) * 0.6, 0.0]) * 0.35e-3
        seg = W.Segment("line", float(rng.uniform(40, 120)), float(rng.uniform(0.6, 1.5)), p0=c - d, p1=c + d)
        out.append(W.sources_from_segments([seg], 2e-6))
    return out


def _pair(monkeypatch, patch, scan, opts):
    from paper_2511_20432_amd import sa_iga
    monkeypatch.setenv("SA_IGA_NO_TENSOR", "1")
    gen = sa_iga.Model(patch, W.MAT_CFG, scan, opts)
    monkeypatch.delenv("SA_IGA_NO_TENSOR")
    ten = sa_iga.Model(patch, W.MAT_CFG, scan, opts)
    return gen, ten


def test_tensor_faces_detected():
    from paper_2511_20432_amd import sa_iga
    scan = W.make_scan(_tracks(1), 1e-5, 5, n_steps=[4])
    blk = sa_iga.Model(W.small_block(), W.MAT_CFG, scan)
    assert blk.info.tensor_faces == 6 and blk.info.generic_points == 0
    ann = W.cfg3()
    m = sa_iga.Model(ann.patch, ann.material, W.make_scan(_tracks(1), 1e-5, 5, n_steps=[2]))
    fo = list(m.info.face_offset)
    sizes = [fo[f + 1] - fo[f] for f in range(6)]
    print("annulus face sizes", sizes, "tensor faces", m.info.tensor_faces, "generic", m.info.generic_points,
          flush=True)
    # the ends of the angular direction (the radial planes at 0 and 90 degrees)
    # are planar grids; the arcs and the annular sectors are not
    assert m.info.tensor_faces == 2
    assert m.info.generic_points == m.info.n_bpts - sizes[0] - sizes[1]


@pytest.mark.parametrize("patch_name", ["small", "cfg1"])
def test_tensor_equals_pairwise_fp64(monkeypatch, patch_name):
    patch = W.small_block() if patch_name == "small" else W.cfg1().patch
    scan = W.make_scan(_tracks(3), 1e-5, 5, n_steps=[30, 22, 30])
    gen, ten = _pair(monkeypatch, patch, scan, W.Options(precision=W.PRECISION_FP64))
    assert gen.info.tensor_faces == 0 and ten.info.tensor_faces == 6
    gen.step(30)
    ten.step(30)
    for p in range(3):
        a, b = gen.boundary_fields(p), ten.boundary_fields(p)
        errs = [rel(x, y) for x, y in zip(b, a)]
        print(f"{patch_name} path {p}: T {errs[0]:.2e} grad {errs[1]:.2e} F {errs[2]:.2e} du {errs[3]:.2e}",
              flush=True)
        assert max(errs) <= 1e-12


def test_tensor_equals_pairwise_fp32_far(monkeypatch):
    scan = W.make_scan(_tracks(2), 1e-5, 5, n_steps=[60, 45])
    opts = W.Options(precision=W.PRECISION_FP32_FAR, tau_near=5e-5)
    gen, ten = _pair(monkeypatch, W.small_block(), scan, opts)
    gen.step(60)
    ten.step(60)
    for p in range(2):
        (Tg, Gg, Fg, ug), (Tt, Gt, Ft, ut) = gen.boundary_fields(p), ten.boundary_fields(p)
        err = float(np.abs(Tt - Tg).max() + np.abs(ut - ug).max())
        print(f"path {p}: FP32 far field, tensor vs pairwise max |dT| <= {err:.2e} K, grad rel {rel(Gt, Gg):.2e}",
              flush=True)
        assert err <= 1e-3
        assert rel(Gt, Gg) <= 1e-5
