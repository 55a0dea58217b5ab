"""Benchmark of the semi-analytical IGA hot path on one MI355X.

A step is one theta-step of the whole path for every scan strategy of the
workload: kernel sum at every boundary quadrature point (T~ and grad T~,
Eqs. 7-8), flux and Dirichlet densities, load-vector and projection gathers
(Eqs. 10-11, 18), Dirichlet projection, theta-scheme right-hand side and
solve (Eq. 20).

Headline (`value`, `ms_per_step`): the learned far-history form with its
audits ("mixed+surrogate") on the held-out batch: 128 scan strategies
(seed 1) on the 4 x 2 x 1 mm cubic block (64 x 32 x 16 elements, 64,512
boundary points), every strategy started at a seeded mid-scan step with a
zeroed state, `--warmup` untimed and `--steps` timed batched steps.  The
FP64 form runs the same window; `speedup_vs_fp64` and `max_err_K_vs_fp64`
compare the two.  `value` counts every switched-on source x boundary point
pair of the timed steps, whether summed or replaced by the network.

Beside it: the seed-0 batch in the FP32 far-field and FP64 forms (same
window rules), the raster scan (one path, all 3,788 steps) in both forms,
the quarter annulus (one path, mid-scan window) in both forms with the
pair-by-pair kernel's rate against its VALU roofline, the small block
(all 150 steps), and the paper's own experiments on the part of Table 2
(single source and contour scan, with the net heat-loss diagnostic along the
top arc beside the values of Tables 3-4).  `cpu_baseline` is the FP64 oracle's kernel sum on sampled
slots of the headline window, on every host core of the process's CPU share
and on one core.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "source×point pairs/s + θ-steps/s; mixed+surrogate vs FP64 GPU at ≤0.5 K err"

# The kernel sum on the faces of the block runs as matrix products on the
# matrix cores: per source x point pair 4 products (T~ and the three gradient
# components) of 2 flops; far pairs in FP32, near pairs in FP64.  Dense
# matrix-core peaks of MI355X:
MFMA_FP32 = 157.3e12
MFMA_FP64 = 78.6e12
FLOPS_PER_PAIR = 8
# The pair-by-pair kernel (curved faces) is bound by VALU issue: 256 compute
# units x 64 lanes x 2.4 GHz lane-operations per second; an FP32 far pair
# takes 9 VALU operations and one v_exp_f32 at a quarter of the VALU rate
# (4 issue slots), an FP64 near pair about 28 FP64 operations (the exponent
# chain and the Cody-Waite exponential), at the full FP64 vector rate.
LANE_OPS = 256 * 64 * 2.4e9
SLOTS_FP32_PAIR = 13
SLOTS_FP64_PAIR = 28
# HBM bytes per sum-stage launch (one k_sum_tensor_far and one
# k_sum_tensor_near launch) from rocprofv3 FETCH_SIZE / WRITE_SIZE per
# dispatch over the headline leg, scaled by the same counters on a 256 MiB
# copy (bench.py --copy-calibration: FETCH x 2.000, WRITE x 1.000); the
# commands and counts are in profiles/k_sum_tensor_far_headline_traffic.md.
# Set to None when the kernels change until the counters are taken again.
K_SUM_TRAFFIC = {"far": {"read_bytes": 76.69e6, "written_bytes": 110.10e6},
                 "near": {"read_bytes": 16.07e6, "written_bytes": 79.92e6}}

WINDOW_START = "each strategy at a seeded step in [0, L - warmup - steps) with a zeroed state (u = T_c, F = 0)"


def _k_sum_traffic():
    """HBM bytes (read + written) of one sum-stage launch, or None."""
    t = K_SUM_TRAFFIC
    if not t:
        return None
    return sum(k["read_bytes"] + k["written_bytes"] for k in t.values())


def _sum_roofline(st, sum_ms):
    """Matrix-core roofline of the sum stage: the algorithmic flops over its
    device time, against the peak of the mix of FP32 (far) and FP64 (near)
    pairs."""
    pairs, near = st["pairs"], st["pairs_near"]
    flops = FLOPS_PER_PAIR * pairs
    t_peak = FLOPS_PER_PAIR * ((pairs - near) / MFMA_FP32 + near / MFMA_FP64)
    if sum_ms <= 0 or flops <= 0:
        return {"bound": "mfma", "achieved": None, "peak": None, "unit": "TFLOP/s", "frac": None}
    t = sum_ms * 1e-3
    return {"bound": "mfma", "achieved": flops / t / 1e12, "peak": flops / t_peak / 1e12, "unit": "TFLOP/s",
            "frac": t_peak / t}


def _valu_roofline(st, sum_ms):
    """VALU roofline of the pair-by-pair sum: pairs per second against the
    issue-slot peak of the mix of FP32 far and FP64 near pairs."""
    pairs, near = st["pairs"], st["pairs_near"]
    t_peak = ((pairs - near) * SLOTS_FP32_PAIR + near * SLOTS_FP64_PAIR) / LANE_OPS
    if sum_ms <= 0 or pairs <= 0:
        return {"bound": "alu", "achieved": None, "peak": None, "unit": "pairs/s", "frac": None}
    t = sum_ms * 1e-3
    return {"bound": "alu", "achieved": pairs / t, "peak": pairs / t_peak, "unit": "pairs/s", "frac": t_peak / t}


def jump_to_steps(model, steps):
    """Put path p at step steps[p] with a zeroed state (u = T_c, F = 0, no
    source field yet): the steps run from there do the full work of a
    mid-scan step (every switched-on source of every path is summed).  Uses
    the checkpoint layout: a 32-byte header, then per path its step (int64),
    its audit state (two int64) and its arrays."""
    blob = bytearray(model.save())
    per = (len(blob) - 32) // len(steps)
    for p, st in enumerate(steps):
        off = 32 + p * per
        blob[off:off + 8] = int(st).to_bytes(8, "little", signed=True)
    model.load(bytes(blob))


def _start_steps(w, span, seed):
    L = w.scan.n_steps.astype(np.int64)
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    return (rng.random(len(L)) * np.maximum(L - span, 0)).astype(np.int64)


def _timed(model, n):
    """Time n steps; the stats carry the pass's bounds on the boot-time clock
    (the clock of the profiler's kernel timestamps)."""
    import torch
    model.reset_stats()
    torch.cuda.synchronize()
    b0 = time.clock_gettime_ns(time.CLOCK_BOOTTIME)
    t0 = time.perf_counter()
    model.step(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = model.stats()
    st["window_ns"] = [b0, time.clock_gettime_ns(time.CLOCK_BOOTTIME)]
    return dt, st


def _window(w, precision, start, warmup, steps, tune=True, **kw):
    """A model of w at the given start steps (zeroed state), tuned, advanced
    `warmup` untimed steps; then `steps` steps timed twice from the same
    state: without per-stage events (the throughput) and with them (stage
    times and kernel-sum launch durations).  The model is left after the
    timed steps."""
    from paper_2511_20432_amd import sa_iga
    from paper_2511_20432_amd import workloads as W
    t0 = time.perf_counter()
    m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=precision, tau_near=2e-4), timing=0, **kw)
    setup_s = time.perf_counter() - t0
    if start is not None:
        jump_to_steps(m, start)
    tuned = m.autotune(reps=2) if tune else None
    if warmup > 0:
        m.step(warmup)
    ck = m.save()
    dt, st = _timed(m, steps)
    final = m.save()
    m.load(ck)
    m.set_timing(True)
    dt_ev, st_ev = _timed(m, steps)
    m.set_timing(False)
    m.load(final)
    st["stage_ms"] = st_ev["stage_ms"]
    st["stage_launches"] = st_ev["stage_launches"]
    st["seconds_with_events"] = dt_ev
    st["window_ns_with_events"] = st_ev["window_ns"]
    st["autotune"] = tuned
    st["setup_s"] = setup_s
    return m, dt, st


def _report(st, dt, steps):
    sum_ms = st["stage_ms"]["sum"]
    covered = st["pairs"] + st["pairs_net"]
    return {
        "pairs_per_s": covered / dt, "pairs_summed_per_s": st["pairs"] / dt,
        "path_steps_per_s": st["steps"] / dt, "ms_per_step": 1e3 * dt / steps,
        "pairs_per_step": covered / steps, "path_steps": st["steps"],
        "sum_gpair_s": st["pairs"] / (sum_ms * 1e-3) / 1e9 if sum_ms > 0 else None,
        "stage_ms_per_step": {k: v / steps for k, v in st["stage_ms"].items()},
        "ms_per_step_with_stage_events": 1e3 * st["seconds_with_events"] / steps,
        "rollbacks": st["rollbacks"], "autotune": st["autotune"], "setup_s": st["setup_s"],
        "host_enqueue_ms_per_step": st["host_enqueue_ms"] / steps,
        "pcg_iterations_per_path_step": st["pcg_iterations"] / max(st["steps"], 1),
        "dirichlet_iterations_per_path_step": st["dirichlet_iterations"] / max(st["steps"], 1),
        "window_boottime_ns": {"plain": st["window_ns"], "with_events": st["window_ns_with_events"]},
    }


def load_point_share(patch):
    """Share of the boundary points whose T~ and grad T~ feed the step: the
    Neumann faces (the load vector, Eq. 18) and the Dirichlet face (its
    data).  The source-plane face's points are summed for the outputs (the
    surface temperature), which the step itself does not use."""
    from paper_2511_20432_amd import workloads as W
    per_face = []
    for f in range(6):
        d = f // 2
        m = [patch.n_elem(k) * patch.quad_face for k in range(3) if k != d]
        per_face.append(m[0] * m[1])
    used = sum(n for f, n in enumerate(per_face) if patch.face_role[f] != W.FACE_SOURCE_PLANE)
    return used / sum(per_face)


def _max_err(a, b):
    """Bound of max |T - T_ref| at the boundary points over all paths:
    |dT~| + max |du| (R_A >= 0 and sum_A R_A = 1 at every point)."""
    worst = 0.0
    for p in range(a.info.n_paths):
        Ta, _, _, ua = a.boundary_fields(p)
        Tb, _, _, ub = b.boundary_fields(p)
        worst = max(worst, float(np.abs(Ta - Tb).max() + np.abs(ua - ub).max()))
    return worst


def train_network(n_train=2_000_000, epochs=4, e_scale=0.1):
    """The far-history network, trained here on the GPU by the library's
    kernels on exact far sums of 64 strategies with seeds 1000..1063."""
    import torch
    from paper_2511_20432_amd import sa_iga, surrogate
    from paper_2511_20432_amd import workloads as W
    t0 = time.perf_counter()
    patch = W.cfg2().patch
    X, T, G = surrogate.training_set(patch, surrogate.strategy_scan(range(1000, 1064)), n_train, e_scale, seed=0)
    ts, gs = surrogate.scales_of(T, G)
    Y = surrogate.targets(T, G, ts, gs)
    del T, G
    net = sa_iga.Mlp(surrogate.init_params(0))
    hist = surrogate.train(net, X, Y, epochs=epochs, batch=4096, lr=1e-3)
    blob = surrogate.weights_blob(net.params(), ts, gs, e_scale)
    del X, Y, net
    torch.cuda.empty_cache()
    info = {"samples": n_train, "epochs": epochs, "loss_per_epoch": hist, "seconds": time.perf_counter() - t0,
            "t_scale_K": ts, "g_scale_K_per_m": gs, "e_scale_J": e_scale, "train_seeds": "1000..1063"}
    return blob, info


def _batch_desc(w, seed):
    return (f"{w.scan.n_paths} scan strategies (seed {seed}) on the 4x2x1 mm block, cubic B-splines 64x32x16, "
            f"64512 boundary points; hatch angle from {{0,45,67,90}} deg, 0.1 mm hatch, power U[40,120] W, "
            f"speed U[0.6,1.5] m/s, lengths U[500,4000] steps (sum {int(w.scan.n_steps.sum())}), "
            f"{len(w.scan.tick)} sources, dt 10 us, 5 sources/step")


def run_headline(warmup, steps, blob):
    """The audited learned far-history form and the FP64 form on the held-out
    batch (seed 1), same window; also the network forced on every step."""
    from paper_2511_20432_amd import workloads as W
    seed = 1
    w = W.cfg4(seed=seed)
    start = _start_steps(w, warmup + steps, seed)
    out = {"workload": _batch_desc(w, seed), "start": WINDOW_START}
    print(f"[bench] headline fp64: {warmup} + {steps} steps of {w.scan.n_paths} strategies", file=sys.stderr,
          flush=True)
    ref, dt, st = _window(w, W.PRECISION_FP64, start, warmup, steps)
    out["fp64"] = _report(st, dt, steps)
    out["fp64"]["sum_roofline"] = _sum_roofline(st, st["stage_ms"]["sum"])
    for form, kw in (("surrogate_audited", {}), ("surrogate_forced", {"audit_tol": 1e30})):
        print(f"[bench] headline {form}", file=sys.stderr, flush=True)
        m, dt, st = _window(w, W.PRECISION_SURROGATE, start, warmup, steps, surrogate_weights=blob, **kw)
        r = _report(st, dt, steps)
        r.update({k: st[k] for k in ("net_steps", "pairs_net", "audits", "audit_failures", "audit_max_err")})
        r["sum_roofline"] = _sum_roofline(st, st["stage_ms"]["sum"])
        r["sum_launches_per_step"] = st["stage_launches"]["sum"] / steps
        r["sum_ms_per_launch"] = (st["stage_ms"]["sum"] / st["stage_launches"]["sum"]
                                  if st["stage_launches"]["sum"] else None)
        net_ms = st["stage_ms"]["net"]
        flops = st["net_steps"] * 64512 * 3 * 2 * 256 * 256
        if net_ms > 0 and flops > 0:
            r["net_roofline"] = {"bound": "mfma", "achieved": flops / (net_ms * 1e-3) / 1e12, "peak": 2500.0,
                                 "unit": "TFLOP/s", "frac": flops / (net_ms * 1e-3) / 2.5e15,
                                 "note": "stage time includes the far-energy bins, first-layer constants and audits"}
        r["max_err_K_vs_fp64"] = _max_err(m, ref)
        r["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / r["ms_per_step"]
        out[form] = r
        m.close()
    ref.close()
    return w, start, out


def run_batch(warmup, steps, seed=0):
    from paper_2511_20432_amd import workloads as W
    w = W.cfg4(seed=seed)
    start = _start_steps(w, warmup + steps, seed)
    out = {"workload": _batch_desc(w, seed), "start": WINDOW_START}
    models = {}
    for form, prec in (("fp32far", W.PRECISION_FP32_FAR), ("fp64", W.PRECISION_FP64)):
        print(f"[bench] batch seed {seed} {form}", file=sys.stderr, flush=True)
        m, dt, st = _window(w, prec, start, warmup, steps)
        out[form] = _report(st, dt, steps)
        out[form]["sum_roofline"] = _sum_roofline(st, st["stage_ms"]["sum"])
        models[form] = m
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32far"]["ms_per_step"]
    out["max_err_K_vs_fp64"] = _max_err(models["fp32far"], models["fp64"])
    for m in models.values():
        m.close()
    return out


def run_raster(warmup):
    """The raster scan, one path: every one of its steps timed, both forms."""
    from paper_2511_20432_amd import sa_iga
    from paper_2511_20432_amd import workloads as W
    w = W.cfg2(seed=0)
    n = int(w.scan.n_steps[0])
    out = {"workload": "raster: 4x2x1 mm block, cubic B-splines 64x32x16, 64512 boundary points, 10 tracks "
                       f"x 0.1 mm hatch, 80 W, 1 m/s, dt 10 us, 5 sources/step, {len(w.scan.tick)} sources, "
                       f"all {n} steps timed from step 0", "steps": n}
    models = {}
    for form, prec in (("fp32far", W.PRECISION_FP32_FAR), ("fp64", W.PRECISION_FP64)):
        print(f"[bench] raster {form}: {n} steps", file=sys.stderr, flush=True)
        if warmup > 0:      # warm-up steps on an object of their own
            m0 = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=prec, tau_near=2e-4))
            m0.step(warmup)
            m0.close()
        m, dt, st = _window(w, prec, None, 0, n)
        out[form] = _report(st, dt, n)
        out[form]["sum_roofline"] = _sum_roofline(st, st["stage_ms"]["sum"])
        models[form] = m
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32far"]["ms_per_step"]
    out["max_err_K_vs_fp64"] = _max_err(models["fp32far"], models["fp64"])
    out["heat_loss_fp64"] = _heat_loss(models["fp64"])
    for m in models.values():
        m.close()
    return out


def _heat_loss(m, faces=(0, 1, 2, 3), top=5):
    """The net heat-loss diagnostic (Sec. 3.1) along the top edge of each
    lateral face at the model's current time: integrals of |q~ + q^| ds and
    |q~| ds (W/m) and their ratio."""
    out = {}
    for f in faces:
        t0 = time.perf_counter()
        r = m.heat_loss(f, top, quad=4)
        out[f"face{f}"] = {"net_W_per_m": r["net"], "tilde_W_per_m": r["tilde"],
                           "ratio": r["net"] / r["tilde"] if r["tilde"] > 0 else None, "points": len(r["ds"]),
                           "ms": 1e3 * (time.perf_counter() - t0)}
    return out


def run_annulus(warmup, steps):
    """The quarter annulus, one path, from the middle of its scan: both forms
    as the library runs them (matrix-core sum on the two planar ends, the
    pair-by-pair kernel on the curved and annular faces), and the FP32
    far-field form with the pair-by-pair kernel on every face for that
    kernel's roofline."""
    from paper_2511_20432_amd import workloads as W
    w = W.cfg3(seed=0)
    n = int(w.scan.n_steps[0])
    s0 = n // 2
    out = {"workload": "quarter annulus r in [2,4] mm x 1 mm, quadratic NURBS 48x24x12, 36288 boundary points; "
                       "contour at r = 3.5 mm then 45 deg hatches, U[60,100] W, 0.8 m/s, dt 10 us, 8 sources/step, "
                       f"{len(w.scan.tick)} sources, {n} steps",
           "start": f"step {s0} with a zeroed state, {warmup} untimed steps", "steps": steps}
    models = {}
    for form, prec in (("fp32far", W.PRECISION_FP32_FAR), ("fp64", W.PRECISION_FP64)):
        print(f"[bench] annulus {form}", file=sys.stderr, flush=True)
        m, dt, st = _window(w, prec, [s0], warmup, steps)
        out[form] = _report(st, dt, steps)
        models[form] = m
    out["speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32far"]["ms_per_step"]
    out["max_err_K_vs_fp64"] = _max_err(models["fp32far"], models["fp64"])
    for m in models.values():
        m.close()
    os.environ["SA_IGA_NO_TENSOR"] = "1"
    try:
        print("[bench] annulus fp32far, pair-by-pair kernel on every face", file=sys.stderr, flush=True)
        m, dt, st = _window(w, W.PRECISION_FP32_FAR, [s0], warmup, steps)
    finally:
        del os.environ["SA_IGA_NO_TENSOR"]
    r = _report(st, dt, steps)
    r["k_sum_roofline"] = _valu_roofline(st, st["stage_ms"]["sum"])
    r["k_sum_roofline"]["kernel"] = "k_sum (pair by pair; far pairs FP32, near pairs FP64)"
    out["fp32far_pair_by_pair"] = r
    m.close()
    return out


def run_small():
    from paper_2511_20432_amd import workloads as W
    w = W.cfg1()
    n = int(w.scan.n_steps[0])
    m, dt, st = _window(w, W.PRECISION_FP64, None, 0, n, tune=False)
    r = _report(st, dt, n)
    r["heat_loss"] = _heat_loss(m)
    m.close()
    r["workload"] = (f"small block 2x1x1 mm, quadratic B-splines 16x8x8, one track, 40 W, 1 m/s, 10 sources/step, "
                     f"all {n} steps, FP64")
    return r


def run_multipatch():
    """A multi-patch part: the three-patch L-shaped part (the corner square
    and two arms, 24 x 24 x 12 quadratic elements per patch), all steps of
    its track through both interfaces, FP64 and FP32 far field (one path,
    pair-by-pair sum, Jacobi CG)."""
    import torch
    from paper_2511_20432_amd import sa_iga
    from paper_2511_20432_amd import workloads as W
    w = W.l_part(n_el=(24, 24, 12))
    n = int(w.scan.n_steps[0])
    ns = w.scan.sources_per_step
    act = np.searchsorted(w.scan.tick, ns * np.arange(1, n + 1), side="right")
    out = {"workload": (f"L-shaped part of three conforming patches (1 mm corner square and two 1 mm arms, "
                        f"0.5 mm high, quadratic, 24x24x12 elements each), one track of {n} steps through both "
                        f"interfaces, 80 W, 1 m/s, 5 sources/step")}
    ref = None
    for name, prec in (("fp64", W.PRECISION_FP64), ("fp32far", W.PRECISION_FP32_FAR)):
        t0 = time.perf_counter()
        m = sa_iga.MultiPatchModel(w.patches, w.maps, w.material, w.scan, W.Options(precision=prec, tau_near=2e-4))
        setup_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.step(n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        info = m.get_info()
        T, _, _, du = m.boundary_fields()
        pairs = float(act.sum()) * info.n_bpts
        r = {"n_dof": info.n_dof, "n_bpts": info.n_bpts, "nnz": info.nnz, "setup_s": setup_s,
             "ms_per_step": 1e3 * dt / n, "pairs_per_s": pairs / dt, "steps": n,
             "cg_iterations_per_step": info.pcg_iterations / n,
             "projection_cg_iterations_per_step": info.dirichlet_iterations / n}
        if ref is None:
            ref = (T, du)
        else:
            r["max_err_K_vs_fp64"] = float(np.abs(T - ref[0]).max() + np.abs(du - ref[1]).max())
        out[name] = r
        m.close()
    return out


# Tables 3 and 4: the paper's integrated net heat-loss rate along the top arc
# (J s^-1 m^-1) and its percentage of the analytical field's, IGA meshes with
# minimum element sizes 100, 68 and 50 um (context: an FEM reference decides
# accuracy there, which is not reproduced)
PAPER_TABLE3_IGA = {"100um": (974.0, 27.64), "68um": (323.0, 9.17), "50um": (167.0, 4.75)}
PAPER_TABLE4_IGA_100UM = {"2ms": (2.41e4, 14.94), "3ms": (1.34e4, 8.03)}


def run_paper_parts():
    """The paper's experiments on the part of Table 2 (s = 2, Ti-6Al-4V), on
    uniformly h-refined quadratic meshes named by their nominal smallest
    element (along the arc): the single source of Sec. 3.1 after 20 steps
    (age 1.9e-4 s) and the contour scan of Sec. 3.2 at 2 and 3 ms, with the
    net heat-loss diagnostic along the top arc."""
    from paper_2511_20432_amd import sa_iga
    from paper_2511_20432_amd import workloads as W
    meshes = {"100um": (8, 10, 20), "68um": (12, 15, 30), "50um": (16, 20, 40)}
    out = {"e1": {}, "e2": {}}
    for name, sp in meshes.items():
        w = W.e1(sp)
        t0 = time.perf_counter()
        m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP64, kernel_scale=2.0))
        t1 = time.perf_counter()
        m.step(20)
        t2 = time.perf_counter()
        r = m.heat_loss(2, 5, quad=4)
        st = m.stats()
        out["e1"][name] = {"splits": sp, "n_dof": m.info.n_dof, "setup_s": t1 - t0, "ms_per_step": 1e3 * (t2 - t1) / 20,
                           "pcg_iterations_per_step": st["pcg_iterations"] / 20,
                           "net_W_per_m": r["net"], "tilde_W_per_m": r["tilde"],
                           "percent": 100 * r["net"] / r["tilde"], "paper_iga": PAPER_TABLE3_IGA[name]}
        m.close()
    for name in ("100um", "50um"):
        sp = meshes[name]
        w = W.e2(sp)
        m = sa_iga.Model(w.patch, w.material, w.scan, W.Options(precision=W.PRECISION_FP64, kernel_scale=2.0))
        res = {"splits": sp, "n_dof": m.info.n_dof}
        done = 0
        step_s = 0.0
        for tag, step in (("2ms", 200), ("3ms", 300)):
            t0 = time.perf_counter()
            m.step(step - done)
            step_s += time.perf_counter() - t0
            done = step
            r = m.heat_loss(2, 5, quad=4)
            res[tag] = {"net_W_per_m": r["net"], "tilde_W_per_m": r["tilde"], "percent": 100 * r["net"] / r["tilde"]}
            if name == "100um" and tag == "3ms":
                # snapshots: the top surface and 50 um below it (Ti-6Al-4V liquidus 1923 K as the threshold)
                from paper_2511_20432_amd import snapshots
                t0s = time.perf_counter()
                for lab, z in (("top", 2e-3), ("50um_below", 2e-3 - 50e-6)):
                    xs, ys, T = snapshots.plane(m, z, (0.0, 0.0), (2e-3, 2e-3), (160, 160))
                    res[f"snapshot_{lab}"] = snapshots.summary(xs, ys, T, 1923.0)
                res["snapshot_seconds"] = time.perf_counter() - t0s
        res["ms_per_step"] = 1e3 * step_s / 300
        res["paper_iga_100um"] = PAPER_TABLE4_IGA_100UM
        out["e2"][name] = res
        m.close()
    return out


def _cpu_model():
    cpu = platform.processor() or platform.machine()
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu


def cpu_baseline(w, start, warmup, n_slots=24, n_slots_1core=2):
    """The oracle's FP64 kernel sum (Eqs. 7-8) at every boundary point for
    sampled slots (strategy, step) of the headline window: the first timed
    step of the first strategies, on every core of the process's CPU share
    and on one core."""
    from oracle import iga, pointsource
    bt = iga.boundary_tables(w.patch)
    x = bt["x"]
    res = {}
    for label, nthr, k in (("all", pointsource.default_threads(), n_slots), ("one", 1, n_slots_1core)):
        pairs = 0
        t0 = time.perf_counter()
        for p in range(k):
            sc = w.scan.path(p)
            s = int(start[p]) + warmup + 1
            pointsource.field(x, sc.xyz, sc.tick, sc.energy, s, sc, w.material, threads=nthr)
            pairs += len(x) * int(np.searchsorted(sc.tick, s * sc.sources_per_step, side="right"))
        res[label] = (pairs, time.perf_counter() - t0, nthr, k)
    pa, ta, na, ka = res["all"]
    p1, t1, _, k1 = res["one"]
    return {"value": pa / ta, "unit": "pairs/s", "cores": na, "kind": "oracle",
            "sample": f"numpy FP64 kernel sum at all {len(x)} boundary points for the first timed step of "
                      f"strategies 0..{ka - 1} of the headline window: {pa:.3e} pairs in {ta:.1f} s on {na} "
                      f"threads ({_cpu_model()}, {os.cpu_count()} logical CPUs on the host)",
            "one_core": {"value": p1 / t1, "unit": "pairs/s", "cores": 1,
                         "sample": f"strategies 0..{k1 - 1}: {p1:.3e} pairs in {t1:.1f} s"}}


def trace_summary(trace_csv, bench_json, leg="headline", form="surrogate_audited"):
    """Markdown table of the kernels a rocprofv3 kernel trace (csv) records
    inside the timed pass (without stage events) of one window of a bench
    line: dispatches whose start lies between the pass's bounds on the
    boot-time clock."""
    import csv
    line = [ln for ln in open(bench_json).read().splitlines() if ln.startswith("{")][-1]
    rep = json.loads(line)[leg][form]
    t0, t1 = rep["window_boottime_ns"]["plain"]
    per = {}
    with open(trace_csv) as f:
        for row in csv.DictReader(f):
            a, b = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
            if t0 <= a <= t1:
                k = row["Kernel_Name"]
                c = per.setdefault(k, [0, 0.0])
                c[0] += 1
                c[1] += (b - a) * 1e-3
    steps = round(1e-6 * (t1 - t0) / rep["ms_per_step"])
    total = sum(v[1] for v in per.values())
    out = [f"Timed pass of `{leg}.{form}` under the profiler: {(t1 - t0) * 1e-6:.1f} ms of wall time, {steps} "
           f"steps, {rep['ms_per_step']:.3f} ms per step in the profiled run's bench line.", "",
           "| kernel | calls | average (us) | per step (us) | share of kernel time |", "|---|---:|---:|---:|---:|"]
    for k, (n, us) in sorted(per.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{k[:70]}` | {n} | {us / n:.1f} | {us / max(steps, 1):.1f} | {100 * us / total:.1f} % |")
    return "\n".join(out)


def graph_probe(kernels=12, reps=2000):
    """Host cost on this system of issuing `kernels` small kernels as stream
    launches and as one replay of a captured HIP graph (torch's graph capture
    of the same elementwise kernels; no memset nodes): microseconds of host
    time per issue of the whole set, and the device-inclusive time per set."""
    import torch
    torch.cuda.set_device(0)
    xs = [torch.zeros(1024, device="cuda") for _ in range(kernels)]

    def issue():
        for x in xs:
            x.add_(1.0)

    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(3):
            issue()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        issue()
    torch.cuda.synchronize()
    out = {}
    for label, fn in (("stream_launches", issue), ("graph_replay", g.replay)):
        with torch.cuda.stream(st):
            for _ in range(50):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            t1 = time.perf_counter()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        out[label] = {"host_us_per_set": 1e6 * (t1 - t0) / reps, "us_per_set_incl_device": 1e6 * (t2 - t0) / reps}
    out["kernels_per_set"] = kernels
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--graph-probe":
        print(json.dumps(graph_probe()))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--trace-summary":
        print(trace_summary(*sys.argv[2:]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60, help="timed batched steps of the headline window")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed ones")
    ap.add_argument("--legs", default="headline,batch,raster,annulus,small,paper,multipatch",
                    help="comma-separated subset of headline,batch,raster,annulus,small,paper,multipatch")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device to device five times (the reference kernel of the HBM "
                         "counter scale) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 5 x 256 MiB", flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the path is not sharded over several GPUs",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "no GPU"
    torch.cuda.set_device(0)
    legs = {s.strip() for s in args.legs.split(",") if s.strip()}
    steps, warmup = max(1, args.steps), max(0, args.warmup)
    out = {}
    if "headline" in legs:
        print("[bench] training the far-history network", file=sys.stderr, flush=True)
        blob, training = train_network()
        w5, start, head = run_headline(warmup, steps, blob)
        head["training"] = training
        a = head["surrogate_audited"]
        roof = dict(a["sum_roofline"])
        roof.update({"traffic": _k_sum_traffic(),
                     "traffic_unit": "HBM bytes per sum-stage launch (read + written)",
                     "kernel": "the matrix-core kernel sum (k_sum_tensor_far: far chunks FP32; k_sum_tensor_near: "
                               "near chunks FP64), the dominant stage of the window",
                     "avg_ms_per_launch": a["sum_ms_per_launch"], "launches_per_step": a["sum_launches_per_step"],
                     "pairs_per_launch": a["pairs_per_step"] / max(a["sum_launches_per_step"], 1e-30)})
        out.update({
            "metric": METRIC, "value": a["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": a["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+f64+bf16", "data": "synthetic",
            "config": {"workload": "learned far-history form with audits on the held-out batch: " + head["workload"]
                       + f"; window: {WINDOW_START}, {warmup} untimed + {steps} timed batched steps",
                       "form": "surrogate_audited (network far field where its audit passed, else FP32 far "
                               "sum; near sources, loads and solves FP64)",
                       "tau_near_s": 2e-4, "theta": 0.5, "audit_every": 50, "audit_frac": 0.01,
                       "audit_tol_K": 0.5, "preconditioner": "fast diagonalisation"},
            "steps_per_s": a["path_steps_per_s"],
            "pairs_feeding_the_step_per_s": a["pairs_per_s"] * load_point_share(w5.patch),
            "speedup_vs_fp64": a["speedup_vs_fp64"], "max_err_K_vs_fp64": a["max_err_K_vs_fp64"],
            "roofline": roof,
            "headline": head,
        })
    if "batch" in legs:
        out["batch"] = run_batch(warmup, steps)
    if "raster" in legs:
        out["raster"] = run_raster(warmup)
    if "annulus" in legs:
        out["annulus"] = run_annulus(warmup, max(steps, 200))
    if "small" in legs:
        out["small"] = run_small()
    if "paper" in legs:
        print("[bench] the paper's experiments on the Table 2 part", file=sys.stderr, flush=True)
        out["paper_parts"] = run_paper_parts()
    if "multipatch" in legs:
        print("[bench] a multi-patch part", file=sys.stderr, flush=True)
        out["multipatch"] = run_multipatch()
    if "headline" in legs and not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle kernel sum)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w5, start, warmup)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
