"""The device-pointer queries of the C ABI (sa_iga_eval_temperature_device,
sa_iga_get_boundary_fields_device) on torch tensors:

  * T and grad T at parametric points, with the basis evaluated on the GPU,
    against the host-table query and the FP64 oracle (1e-9 normwise, as the
    host query), on the block and on the rational quarter annulus (curved
    NURBS weights); points outside [0,1]^3 give NaN;
  * the boundary fields copied device to device equal the host copies
    bitwise;
  * both run on the stream the object was given (a torch side stream).
"""
import numpy as np
import pytest
import torch

from oracle import solver
from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _points(seed, n=200):
    rng = np.random.default_rng(seed)
    xi = rng.random((n, 3))
    xi[:20, 2] = 1.0                  # on the top face
    xi[20:30] = [0.0, 0.0, 0.0]       # a corner
    xi[30:40] = [1.0, 1.0, 1.0]       # the opposite corner (right ends of the knot vectors)
    xi[40:50, 0] = 0.5                # on an interior knot plane
    return xi


def _device(gm, xi):
    T, G = gm.eval_temperature_device(torch.from_numpy(xi).cuda())
    torch.cuda.synchronize()
    return T.cpu().numpy(), G.cpu().numpy()


def test_eval_temperature_device_matches_host_and_oracle():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg1()
    gm = sa_iga.Model(w.patch, w.material, w.scan)
    om = solver.Model(w.patch, w.material, w.scan)
    gm.step(40)
    om.advance(40)
    xi = _points(7)
    Td, Gd = _device(gm, xi)
    Th, Gh = gm.eval_temperature(xi)
    Tr, Gr, _ = om.evaluate(xi)
    T0 = w.material.T0
    print(f"device vs host: T {rel(Td - T0, Th - T0):.2e}, grad {rel(Gd, Gh):.2e}; "
          f"vs oracle: T {rel(Td - T0, Tr - T0):.2e}, grad {rel(Gd, Gr):.2e}", flush=True)
    assert rel(Td - T0, Th - T0) <= 1e-12 and rel(Gd, Gh) <= 1e-12
    assert rel(Td - T0, Tr - T0) <= TOL64 and rel(Gd, Gr) <= TOL64
    # without the gradient, and outside the unit cube: NaN
    T1, G1 = gm.eval_temperature_device(torch.tensor([[0.5, 0.5, 1.5], [-0.1, 0.2, 0.3], [0.3, 0.4, 1.0]],
                                                      dtype=torch.float64, device="cuda"), gradient=False)
    torch.cuda.synchronize()
    T1 = T1.cpu().numpy()
    assert G1 is None and np.isnan(T1[0]) and np.isnan(T1[1])
    assert T1[2] == pytest.approx(gm.eval_temperature(np.array([[0.3, 0.4, 1.0]]))[0][0], rel=1e-12)


def test_eval_temperature_device_on_the_rational_annulus():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg3(n_el=(12, 6, 4), options=W.Options(precision=W.PRECISION_FP64))
    gm = sa_iga.Model(w.patch, w.material, w.scan, w.options)
    gm.step(30)
    xi = _points(11, 300)
    Td, Gd = _device(gm, xi)
    Th, Gh = gm.eval_temperature(xi)
    T0 = w.material.T0
    print(f"annulus device vs host: T {rel(Td - T0, Th - T0):.2e}, grad {rel(Gd, Gh):.2e}", flush=True)
    assert np.abs(Th - T0).max() > 1.0
    assert rel(Td - T0, Th - T0) <= 1e-12 and rel(Gd, Gh) <= 1e-12


def test_boundary_fields_device_equal_host_copies_on_a_side_stream():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg1()
    gm = sa_iga.Model(w.patch, w.material, w.scan)
    side = torch.cuda.Stream()
    gm.set_stream(side.cuda_stream)
    gm.step(25)
    with torch.cuda.stream(side):
        Td, Gd, Fd, ud = gm.boundary_fields_device()
        xi = torch.from_numpy(_points(5, 50)).cuda()
        side.synchronize()
        Te, Ge = gm.eval_temperature_device(xi)
    side.synchronize()
    T, G, F, u = gm.boundary_fields()
    assert np.array_equal(Td.cpu().numpy(), T) and np.array_equal(Gd.cpu().numpy().T, G)
    assert np.array_equal(Fd.cpu().numpy(), F) and np.array_equal(ud.cpu().numpy(), u)
    Th, Gh = gm.eval_temperature(xi.cpu().numpy())
    T0 = w.material.T0
    assert rel(Te.cpu().numpy() - T0, Th - T0) <= 1e-12 and rel(Ge.cpu().numpy(), Gh) <= 1e-12
    gm.set_stream(None)
