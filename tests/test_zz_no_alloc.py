"""The allocation-free source-field evaluation (sa_iga_eval_source_field_noalloc,
for callers that cannot allocate device memory) against the allocating
entry point sa_iga_eval_source_field, through the C ABI: T~ and grad T~
(Eqs. 7-8) at query points, two calls in a row with the second smaller, in
the FP64 and FP32 far-field forms, on a history long enough that the chunk
count is capped, and the size limits."""
import numpy as np
import pytest
import torch

from paper_2511_20432_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


def rel(a, b):
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / max(np.abs(b).max(), 1e-300))


def _points(patch, n, seed):
    ctrl = patch.ctrl.reshape(-1, 4)[:, :3]
    lo, hi = ctrl.min(axis=0), ctrl.max(axis=0)
    rng = np.random.default_rng(seed)
    return lo + rng.random((n, 3)) * (hi - lo)


def _compare(m, x, step, label):
    T_h, G_h = m.source_field(x, step)                    # G_h [n, 3]
    xd = torch.from_numpy(x).cuda()
    T_d, G_d = m.source_field_noalloc(xd, step)
    torch.cuda.synchronize()
    T_d, G_d = T_d.cpu().numpy(), G_d.cpu().numpy().T
    e_T, e_G = rel(T_d, T_h), rel(G_d, G_h)
    print(f"{label}: n {len(x)}, step {step}: T rel {e_T:.2e}, grad rel {e_G:.2e}, max T {np.abs(T_h).max():.3e}",
          flush=True)
    assert np.abs(T_h).max() > 0
    assert e_T <= TOL and e_G <= TOL
    return T_d


@pytest.mark.parametrize("prec", [W.PRECISION_FP64, W.PRECISION_FP32_FAR])
def test_two_calls_second_smaller_match_allocating_call(prec):
    from paper_2511_20432_amd import sa_iga
    w = W.cfg1()
    m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=prec, tau_near=2e-5))
    m.step(120)
    x1 = _points(w.patch, 4096, 1)
    x2 = _points(w.patch, 777, 2)
    _compare(m, x1, 120, "first call")
    _compare(m, x2, 37, "second call")
    # the second call's outputs do not depend on what the first left behind
    xd = torch.from_numpy(x2).cuda()
    a, _ = m.source_field_noalloc(xd, 37)
    torch.cuda.synchronize()
    _compare(m, x1[:1000], 90, "third call")
    b, _ = m.source_field_noalloc(xd, 37, grad=False)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    m.close()


@pytest.mark.parametrize("prec", [W.PRECISION_FP64, W.PRECISION_FP32_FAR])
def test_long_history_with_capped_chunks(prec):
    """15,000 switched-on sources of the raster scan: the allocating call
    splits them into more than 64 chunks, the allocation-free one into at
    most 64, so the two agree to rounding."""
    from paper_2511_20432_amd import sa_iga
    w = W.cfg2(seed=0)
    m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=prec, tau_near=2e-4))
    x = _points(w.patch, 4096, 3)
    x[:, 2] = 1e-3 - np.abs(x[:, 2] - 1e-3) * 0.05        # most points near the top surface
    _compare(m, x, 3000, "raster history")
    _compare(m, x[:64], 1500, "raster history, 64 points")
    m.close()


def test_size_limits():
    from paper_2511_20432_amd import sa_iga
    w = W.cfg1()
    m = sa_iga.Model(w.patch, w.material, w.scan, W.Options())
    x = torch.zeros((4097, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(sa_iga.SaError) as e:
        m.source_field_noalloc(x, 10)
    assert "4096" in str(e.value)
    T, G = m.source_field_noalloc(x[:0], 10)
    torch.cuda.synchronize()
    assert T.numel() == 0
    m.close()
