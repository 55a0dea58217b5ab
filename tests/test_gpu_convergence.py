"""The paper's accuracy study (Sec. 3.1: the relative error e_r of T^ at a
point near the boundary against the ratio l_e of the element size to the
spot radius), with the exact solution of a rectangular block (the image
lattice: even images across the adiabatic faces, odd across the Dirichlet
bottom) as the reference that the paper took from a fine FEM run.  One
source 100 um from the face x = 0, Ti-6Al-4V, after 20 steps (age 1.9e-4 s);
the probe lies on that face, on the top surface, next to the source.  e_r
falls as the GPU's quadratic meshes are refined (the oracle gives 46 %, 10 %
and 0.55 % for 200, 100 and 50 um elements)."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import closed_forms as cf  # noqa: E402
from paper_2511_20432_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

SIZE = (0.8e-3, 0.8e-3, 0.4e-3)
SRC = (0.1e-3, 0.4e-3, 0.4e-3)
PROBE = (0.0, 0.4e-3, 0.4e-3)
MAT = W.MAT_TI64


def _exact_that(age):
    """T^ - T_c of the block at the probe: the non-identity images of the
    source (s = 2), from the kernel of Eq. 8 with the spot shift."""
    a = MAT.k / (MAT.rho * MAT.cp)
    D = age + (20e-6) ** 2 / (8 * a)
    total = 0.0
    for pos, sg in cf.image_lattice(SRC, SIZE, n_img=2)[1:]:
        r2 = sum((PROBE[i] - pos[i]) ** 2 for i in range(3))
        total += sg * 2.0 * W.E_PAPER / (MAT.rho * MAT.cp * (4 * math.pi * a * D) ** 1.5) * math.exp(-r2 / (4 * a * D))
    return total


def test_error_falls_with_element_size():
    from paper_2511_20432_amd import sa_iga
    scan = W.make_scan([(np.array([SRC]), np.array([1], np.int64), np.array([W.E_PAPER]))], 1e-5, 1, n_steps=[20])
    ref = _exact_that(19 * 1e-5)
    errs = []
    for n in (4, 8, 16):
        patch = W.block_patch((0, 0, 0), SIZE, (n, n, n // 2), 2)
        m = sa_iga.Model(patch, MAT, scan, W.Options(kernel_scale=2.0))
        m.step(20)
        # T^ at the probe: T - T~ (the source field at the probe itself)
        T, _, _ = m.eval_temperature_at(np.array([PROBE]))
        Tt, _ = m.source_field(np.array([PROBE]), 20)
        that = float(T[0] - Tt[0] - MAT.T0)
        le = (SIZE[0] / n) / 20e-6
        errs.append(abs(that - ref) / ref)
        print(f"l_e = {le:.1f} ({SIZE[0] / n * 1e6:.0f} um elements, {m.info.n_dof} DOFs): T^ = {that:.3f} K, "
              f"exact {ref:.3f} K, e_r = {100 * errs[-1]:.2f} %", flush=True)
        m.close()
    assert errs[2] < errs[1] < errs[0] and errs[2] < 0.02
