"""Write the oracle's full-size trajectory snapshots used by the GPU parity
tests of the raster block (cfg2) and the quarter annulus (cfg3).

Calls only the FP64 oracle (oracle/) and the seeded input generators.  The
oracle advances one path from w^0 = 0 through every theta-step (Eq. 20 with
the load vector of Eq. 18 and the Dirichlet projection of Eq. 11), with the
kernel sum of Eqs. 7-8 over every switched-on source at every lateral and
bottom boundary point, and stores the control values w = u - T_c and the
load vector F at the listed steps.

    python tests/golden/make_trajectory_snapshots.py cfg2   # every step (3,788), about 1.5 h on 8 cores
    python tests/golden/make_trajectory_snapshots.py cfg3   # first 2,000 steps

Output: tests/golden/traj_<name>.npz with arrays steps [k], w [k][n_dof],
F [k][n_dof] (FP64), and a text line of what was run in `recipe`.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import solver  # noqa: E402
from paper_2511_20432_amd import workloads as W  # noqa: E402

SNAPSHOTS = {
    "cfg2": (500, 1900, 3788),
    "cfg3": (700, 2000),
}


def workload(name):
    return W.cfg2(seed=0) if name == "cfg2" else W.cfg3(seed=0)


def main(name):
    steps = SNAPSHOTS[name]
    w = workload(name)
    t0 = time.time()
    m = solver.Model(w.patch, w.material, w.scan)
    print(f"[{name}] set-up {time.time() - t0:.0f} s, n_dof {w.patch.n_dof}, "
          f"{len(w.scan.tick)} sources, {int(w.scan.n_steps[0])} steps", flush=True)
    out_w, out_F = [], []
    t0 = time.time()
    for s in steps:
        while m.step < s:
            m.advance(1)
            if m.step % 100 == 0:
                print(f"[{name}] step {m.step} ({time.time() - t0:.0f} s)", flush=True)
        out_w.append(m.w.copy())
        out_F.append(m.F.copy())
    path = os.path.join(HERE, f"traj_{name}.npz")
    recipe = (f"oracle.solver.Model({w.name}, seed 0, theta 0.5, kernel scale 1), "
              f"FP64 kernel sum over all switched-on sources, sparse LU solve; steps {list(steps)}")
    np.savez(path, steps=np.asarray(steps, np.int64), w=np.asarray(out_w), F=np.asarray(out_F),
             recipe=np.asarray(recipe))
    print(f"[{name}] wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["cfg2", "cfg3"]:
        main(n)
