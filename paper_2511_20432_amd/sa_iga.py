"""ctypes binding of libsa_iga.so (include/sa_iga.h).

Argument marshalling only: every step of the model runs in the library's
HIP kernels.  The functions keep the C names; `Model` is a small owner of a
handle for convenience.  Loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import workloads as W

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libsa_iga.so")

SA_OK, SA_EINVAL, SA_ENOMEM, SA_EDEVICE, SA_ENOCONV, SA_ERANGE, SA_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SA_OK", -1: "SA_EINVAL", -2: "SA_ENOMEM", -3: "SA_EDEVICE", -4: "SA_ENOCONV",
                -5: "SA_ERANGE", -6: "SA_ESTATE"}
STAGES = ["coeff", "sum", "reduce", "load", "dirichlet", "rhs", "pcg", "net"]

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


class sa_patch(C.Structure):
    _fields_ = [("degree", C.c_int32 * 3), ("n_ctrl", C.c_int32 * 3), ("knots", _dp * 3),
                ("ctrl_xyzw", _dp), ("face_role", C.c_int32 * 6), ("quad_vol", C.c_int32 * 3),
                ("quad_face", C.c_int32)]


class sa_material(C.Structure):
    _fields_ = [("k", C.c_double), ("rho", C.c_double), ("cp", C.c_double), ("T0", C.c_double)]


class sa_solver_options(C.Structure):
    _fields_ = [("theta", C.c_double), ("kernel_scale", C.c_double), ("precision", C.c_int32),
                ("tau_near", C.c_double), ("pcg_rtol", C.c_double), ("pcg_max_iter", C.c_int32),
                ("preconditioner", C.c_int32), ("timing", C.c_int32), ("points_per_lane", C.c_int32),
                ("waves_per_group", C.c_int32), ("chunk_sources", C.c_int32),
                ("surrogate_weights", C.POINTER(C.c_float)), ("surrogate_len", C.c_int64),
                ("audit_every", C.c_int32), ("audit_frac", C.c_double), ("audit_tol", C.c_double)]


class sa_scan_path(C.Structure):
    _fields_ = [("n_paths", C.c_int32), ("src_offset", _i64p), ("xyz", _dp), ("tick", _i64p),
                ("energy", _dp), ("n_steps", _i32p), ("dt", C.c_double), ("sources_per_step", C.c_int32),
                ("spot_radius", C.c_double), ("opt", C.POINTER(sa_solver_options))]


class sa_info(C.Structure):
    _fields_ = [("n_ctrl", C.c_int32 * 3), ("n_dof", C.c_int64), ("n_bpts", C.c_int64),
                ("face_offset", C.c_int64 * 7), ("n_paths", C.c_int32), ("n_sources", C.c_int64),
                ("n_dirichlet", C.c_int64), ("tensor_faces", C.c_int32), ("generic_points", C.c_int64),
                ("blocked_steps", C.c_int32), ("sum_groups_per_cu_batch", C.c_int32), ("block_lds_pad", C.c_int32),
                ("batch_lds_pad", C.c_int32)]


class sa_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("pairs", C.c_int64), ("pairs_near", C.c_int64),
                ("pcg_iterations", C.c_int64), ("pcg_last_iterations", C.c_int32),
                ("pcg_last_relres", C.c_double), ("dirichlet_iterations", C.c_int64),
                ("stage_ms", C.c_double * 8), ("stage_launches", C.c_int64 * 8),
                ("net_steps", C.c_int64), ("pairs_net", C.c_int64), ("audits", C.c_int64),
                ("audit_failures", C.c_int64), ("audit_max_err", C.c_double), ("rollbacks", C.c_int64),
                ("host_enqueue_ms", C.c_double)]


class sa_mp_info(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("n_paths", C.c_int32), ("n_dof", C.c_int64), ("n_bpts", C.c_int64),
                ("n_dirichlet", C.c_int64), ("n_free", C.c_int64), ("nnz", C.c_int64), ("step", C.c_int64),
                ("n_steps", C.c_int64), ("pcg_iterations", C.c_int64), ("dirichlet_iterations", C.c_int64),
                ("pcg_last_relres", C.c_double)]


EXPORTS = {
    "sa_iga_default_options": (C.c_int, [C.POINTER(sa_solver_options)]),
    "sa_iga_setup": (C.c_int, [C.POINTER(sa_patch), C.POINTER(sa_material), C.POINTER(sa_scan_path),
                               C.POINTER(C.c_void_p)]),
    "sa_iga_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "sa_iga_get_step": (C.c_int, [C.c_void_p, C.c_int32, _i64p]),
    "sa_iga_eval_temperature": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, _dp, _dp, _dp]),
    "sa_iga_get_boundary_fields": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp]),
    "sa_iga_get_boundary_points": (C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    "sa_iga_apply_operator": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp]),
    "sa_iga_eval_source_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, _dp, _dp, _dp]),
    "sa_iga_eval_source_field_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p,
                                                   C.c_void_p, C.c_void_p]),
    "sa_iga_eval_temperature_at": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, _dp, _dp, _dp, _dp]),
    "sa_iga_eval_temperature_device": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_void_p,
                                                 C.c_void_p]),
    "sa_iga_get_boundary_fields_device": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                                    C.c_void_p]),
    "sa_iga_heat_loss": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _i64p, _dp, _dp, _dp,
                                   _dp, _dp, _dp]),
    "sa_iga_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double)]),
    "sa_iga_set_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "sa_iga_get_info": (C.c_int, [C.c_void_p, C.POINTER(sa_info)]),
    "sa_iga_get_stats": (C.c_int, [C.c_void_p, C.POINTER(sa_stats)]),
    "sa_iga_reset_stats": (C.c_int, [C.c_void_p]),
    "sa_iga_save": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    "sa_iga_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "sa_iga_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sa_iga_far_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_void_p, C.c_void_p,
                                   C.c_void_p]),
    "sa_mlp_n_params": (C.c_int64, []),
    "sa_mlp_create": (C.c_int, [C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_void_p)]),
    "sa_mlp_get_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_int64]),
    "sa_mlp_forward": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "sa_mlp_gradients": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.POINTER(C.c_float),
                                   C.POINTER(C.c_double)]),
    "sa_mlp_train_step": (C.c_int, [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_float,
                                    C.POINTER(C.c_double)]),
    "sa_mlp_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sa_mlp_destroy": (None, [C.c_void_p]),
    "sa_mp_setup": (C.c_int, [C.POINTER(sa_patch), C.c_int32, _i64p, C.POINTER(sa_material),
                              C.POINTER(sa_scan_path), C.POINTER(C.c_void_p)]),
    "sa_mp_step": (C.c_int, [C.c_void_p, C.c_int32]),
    "sa_mp_get_info": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(sa_mp_info)]),
    "sa_mp_get_boundary_fields": (C.c_int, [C.c_void_p, C.c_int32, _dp, _dp, _dp, _dp]),
    "sa_mp_get_boundary_points": (C.c_int, [C.c_void_p, _dp, _dp, _dp]),
    "sa_mp_eval_temperature": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, _dp, _dp, _dp]),
    "sa_mp_eval_temperature_at": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, _dp, _dp, _dp, _i32p, _dp]),
    "sa_mp_heat_loss": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _i64p, _dp, _dp, _dp, _dp,
                                  _dp, _dp]),
    "sa_mp_destroy": (None, [C.c_void_p]),
    "sa_iga_last_error": (C.c_char_p, []),
    "sa_iga_destroy": (None, [C.c_void_p]),
}

_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load_library() -> C.CDLL:
    """Load libsa_iga.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} not found: build it with paper_2511_20432_amd.build.build()")
    lib = C.CDLL(_LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int):
    if code != SA_OK:
        raise SaError(code, load_library().sa_iga_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def default_options() -> sa_solver_options:
    o = sa_solver_options()
    check(load_library().sa_iga_default_options(C.byref(o)))
    return o


def _patch_struct(patch: W.Patch, keep) -> sa_patch:
    p = sa_patch()
    for d in range(3):
        p.degree[d] = patch.degree[d]
        p.n_ctrl[d] = patch.n_ctrl[d]
        p.knots[d] = _ptr(keep(patch.knots[d], np.float64), C.c_double)
        p.quad_vol[d] = patch.quad_vol[d]
    p.ctrl_xyzw = _ptr(keep(patch.ctrl, np.float64), C.c_double)
    for f in range(6):
        p.face_role[f] = patch.face_role[f]
    p.quad_face = patch.quad_face
    return p


def _options_struct(options: Optional[W.Options], overrides: dict, keep) -> sa_solver_options:
    o = default_options()
    if options is not None:
        o.theta = options.theta
        o.kernel_scale = options.kernel_scale
        o.precision = options.precision
        o.tau_near = options.tau_near
        o.pcg_rtol = options.pcg_rtol
        o.pcg_max_iter = options.pcg_max_iter
        o.preconditioner = options.preconditioner
    overrides = dict(overrides)
    weights = overrides.pop("surrogate_weights", None)
    if weights is not None:
        weights = keep(weights, np.float32)
        o.surrogate_weights = _ptr(weights, C.c_float)
        o.surrogate_len = len(weights)
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def _scan_struct(scan: W.ScanPath, o: sa_solver_options, keep) -> sa_scan_path:
    s = sa_scan_path()
    s.n_paths = scan.n_paths
    s.src_offset = _ptr(keep(scan.src_offset, np.int64), C.c_int64)
    s.xyz = _ptr(keep(scan.xyz.reshape(-1, 3) if len(scan.xyz) else np.zeros((1, 3)), np.float64), C.c_double)
    s.tick = _ptr(keep(scan.tick if len(scan.tick) else np.ones(1, np.int64), np.int64), C.c_int64)
    s.energy = _ptr(keep(scan.energy if len(scan.energy) else np.zeros(1), np.float64), C.c_double)
    s.n_steps = _ptr(keep(scan.n_steps, np.int32), C.c_int32)
    s.dt = scan.dt
    s.sources_per_step = scan.sources_per_step
    s.spot_radius = scan.spot_radius
    s.opt = C.pointer(o)
    return s


class Model:
    """Owner of one sa_iga handle built from a workload description."""

    def __init__(self, patch: W.Patch, material: W.Material, scan: W.ScanPath,
                 options: Optional[W.Options] = None, **opt_overrides):
        lib = load_library()
        self._lib = lib
        self._keep = []

        def keep(a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            self._keep.append(a)
            return a

        p = _patch_struct(patch, keep)
        m = sa_material(material.k, material.rho, material.cp, material.T0)
        o = _options_struct(options, opt_overrides, keep)
        self.options = o
        s = _scan_struct(scan, o, keep)
        h = C.c_void_p()
        check(lib.sa_iga_setup(C.byref(p), C.byref(m), C.byref(s), C.byref(h)))
        self._keep = []
        self.h = h
        self.T0 = material.T0
        self.info = self.get_info()

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self._lib.sa_iga_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls -----------------------------------------------------------------
    def step(self, n: int = 1):
        check(self._lib.sa_iga_step(self.h, n))

    def get_step(self, path: int = 0) -> int:
        s = C.c_int64()
        check(self._lib.sa_iga_get_step(self.h, path, C.byref(s)))
        return s.value

    def get_info(self) -> sa_info:
        i = sa_info()
        check(self._lib.sa_iga_get_info(self.h, C.byref(i)))
        return i

    def stats(self) -> dict:
        s = sa_stats()
        check(self._lib.sa_iga_get_stats(self.h, C.byref(s)))
        d = {k: getattr(s, k) for k, _ in sa_stats._fields_ if k not in ("stage_ms", "stage_launches")}
        d["stage_ms"] = {STAGES[i]: s.stage_ms[i] for i in range(8)}
        d["stage_launches"] = {STAGES[i]: s.stage_launches[i] for i in range(8)}
        return d

    def reset_stats(self):
        check(self._lib.sa_iga_reset_stats(self.h))

    def set_timing(self, on: bool):
        check(self._lib.sa_iga_set_timing(self.h, 1 if on else 0))

    def autotune(self, reps: int = 3) -> dict:
        """Pick the kernel-sum tile shape with the fastest whole steps (timed
        from mid-scan, state restored); results stay bitwise the same."""
        p, w, ms = C.c_int32(), C.c_int32(), C.c_double()
        check(self._lib.sa_iga_autotune(self.h, reps, C.byref(p), C.byref(w), C.byref(ms)))
        self.info = self.get_info()
        return {"points_per_lane": p.value, "waves_per_group": w.value, "ms_per_step": ms.value,
                "sum_groups_per_cu_batch": self.info.sum_groups_per_cu_batch,
                "batch_lds_pad": self.info.batch_lds_pad, "block_lds_pad": self.info.block_lds_pad,
                "blocked_steps": self.info.blocked_steps}

    def boundary_fields(self, path: int = 0):
        """T~ [nq], grad T~ [nq, 3] at the boundary points, F [n_dof] and
        du [n_dof] = T^ - T_c at the control points."""
        nq, nd = self.info.n_bpts, self.info.n_dof
        T = np.empty(nq)
        G = np.empty((3, nq))
        F = np.empty(nd)
        u = np.empty(nd)
        check(self._lib.sa_iga_get_boundary_fields(self.h, path, _ptr(T, C.c_double), _ptr(G, C.c_double),
                                                   _ptr(F, C.c_double), _ptr(u, C.c_double)))
        return T, G.T.copy(), F, u

    def boundary_points(self):
        nq = self.info.n_bpts
        x = np.empty((nq, 3))
        n = np.empty((nq, 3))
        w = np.empty(nq)
        check(self._lib.sa_iga_get_boundary_points(self.h, _ptr(x, C.c_double), _ptr(n, C.c_double),
                                                   _ptr(w, C.c_double)))
        return x, n, w

    def apply_operator(self, which: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty_like(x)
        check(self._lib.sa_iga_apply_operator(self.h, which, _ptr(x, C.c_double), _ptr(y, C.c_double)))
        return y

    def source_field(self, x: np.ndarray, step: int, path: int = 0):
        x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        n = len(x)
        T = np.empty(n)
        G = np.empty((3, n))
        check(self._lib.sa_iga_eval_source_field(self.h, path, step, n, _ptr(x, C.c_double),
                                                 _ptr(T, C.c_double), _ptr(G, C.c_double)))
        return T, G.T.copy()

    def source_field_noalloc(self, x, step: int, path: int = 0, T=None, grad=None):
        """sa_iga_eval_source_field_noalloc on device tensors: x [n, 3]
        float64; T [n] and grad [3, n] float64 device tensors are allocated
        here when not given (grad=False: none).  The work is enqueued on the
        object's stream; synchronise before reading T or grad."""
        import torch
        assert x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
        n = x.shape[0]
        if T is None:
            T = torch.empty(n, dtype=torch.float64, device=x.device)
        if grad is None:
            grad = torch.empty((3, n), dtype=torch.float64, device=x.device)
        gp = None if grad is False else C.c_void_p(grad.data_ptr())
        check(self._lib.sa_iga_eval_source_field_noalloc(self.h, path, step, n, C.c_void_p(x.data_ptr()),
                                                         C.c_void_p(T.data_ptr()), gp))
        return T, (None if grad is False else grad)

    def eval_temperature_at(self, x: np.ndarray, path: int = 0):
        """T, grad T and the parametric points at physical points x [n, 3]
        (NaN outside the patch)."""
        x = np.ascontiguousarray(x, np.float64).reshape(-1, 3)
        n = len(x)
        T, G, xi = np.empty(n), np.empty((n, 3)), np.empty((n, 3))
        check(self._lib.sa_iga_eval_temperature_at(self.h, path, n, _ptr(x, C.c_double), _ptr(T, C.c_double),
                                                   _ptr(G, C.c_double), _ptr(xi, C.c_double)))
        return T, G, xi

    def heat_loss(self, face: int, edge_face: int, quad: int = 4, path: int = 0) -> dict:
        """Net heat-loss rate along the edge where `face` meets `edge_face`:
        points x, outward normals n, arc-length weights ds, q_tilde, q_hat
        and the integrals of |q~ + q^| ds (net) and |q~| ds (tilde)."""
        n = C.c_int64(0)
        check(self._lib.sa_iga_heat_loss(self.h, path, face, edge_face, quad, C.byref(n), None, None, None, None,
                                         None, None))
        x, nrm = np.empty((n.value, 3)), np.empty((n.value, 3))
        ds, qt, qh, integ = np.empty(n.value), np.empty(n.value), np.empty(n.value), np.empty(2)
        check(self._lib.sa_iga_heat_loss(self.h, path, face, edge_face, quad, C.byref(n), _ptr(x, C.c_double),
                                         _ptr(nrm, C.c_double), _ptr(ds, C.c_double), _ptr(qt, C.c_double),
                                         _ptr(qh, C.c_double), _ptr(integ, C.c_double)))
        return {"x": x, "n": nrm, "ds": ds, "q_tilde": qt, "q_hat": qh, "net": float(integ[0]),
                "tilde": float(integ[1])}

    def eval_temperature(self, xi: np.ndarray, path: int = 0):
        xi = np.ascontiguousarray(xi, np.float64).reshape(-1, 3)
        n = len(xi)
        T = np.empty(n)
        G = np.empty((n, 3))
        check(self._lib.sa_iga_eval_temperature(self.h, path, n, _ptr(xi, C.c_double), _ptr(T, C.c_double),
                                                _ptr(G, C.c_double)))
        return T, G

    def eval_temperature_device(self, xi, path: int = 0, gradient: bool = True):
        """sa_iga_eval_temperature_device on device tensors: xi [n, 3]
        float64 (contiguous); returns T [n] and grad [n, 3] (None when
        gradient is False) as new device tensors.  The work is enqueued on
        the object's stream; synchronise before reading them."""
        import torch
        assert xi.is_cuda and xi.dtype == torch.float64 and xi.is_contiguous() and xi.dim() == 2
        n = xi.shape[0]
        T = torch.empty(n, dtype=torch.float64, device=xi.device)
        G = torch.empty((n, 3), dtype=torch.float64, device=xi.device) if gradient else None
        check(self._lib.sa_iga_eval_temperature_device(self.h, path, n, C.c_void_p(xi.data_ptr()),
                                                       C.c_void_p(T.data_ptr()),
                                                       C.c_void_p(G.data_ptr()) if gradient else None))
        return T, G

    def boundary_fields_device(self, path: int = 0):
        """sa_iga_get_boundary_fields_device into new device tensors: T~ [nq],
        grad T~ [3, nq], F [n_dof], du [n_dof], enqueued on the object's
        stream; synchronise before reading them."""
        import torch
        nq, nd = self.info.n_bpts, self.info.n_dof
        kw = {"dtype": torch.float64, "device": "cuda"}
        T, G, F, u = torch.empty(nq, **kw), torch.empty((3, nq), **kw), torch.empty(nd, **kw), torch.empty(nd, **kw)
        check(self._lib.sa_iga_get_boundary_fields_device(self.h, path, *(C.c_void_p(t.data_ptr())
                                                                          for t in (T, G, F, u))))
        return T, G, F, u

    def save(self) -> bytes:
        n = C.c_size_t(0)
        check(self._lib.sa_iga_save(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        check(self._lib.sa_iga_save(self.h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        check(self._lib.sa_iga_load(self.h, buf, len(blob)))

    def set_stream(self, stream_handle: Optional[int]):
        check(self._lib.sa_iga_set_stream(self.h, C.c_void_p(stream_handle) if stream_handle else None))

    def far_field(self, step: int, e_scale: float, path: int = 0):
        """Exact far field at every boundary point and the network inputs, as
        device tensors: X [n_bpts, 70] float32, T [n_bpts], G [3, n_bpts] float64."""
        import torch
        nq = self.info.n_bpts
        X = torch.empty((nq, 70), dtype=torch.float32, device="cuda")
        T = torch.empty(nq, dtype=torch.float64, device="cuda")
        G = torch.empty((3, nq), dtype=torch.float64, device="cuda")
        torch.cuda.current_stream().synchronize()
        check(self._lib.sa_iga_far_field(self.h, path, step, e_scale, C.c_void_p(X.data_ptr()),
                                         C.c_void_p(T.data_ptr()), C.c_void_p(G.data_ptr())))
        return X, T, G


def _dev(t):
    """Device pointer of a contiguous CUDA tensor (torch's work on it finished)."""
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


class Mlp:
    """Owner of one sa_mlp handle (the far-history network trainer)."""

    def __init__(self, params: np.ndarray):
        lib = load_library()
        self._lib = lib
        p = np.ascontiguousarray(params, dtype=np.float32)
        h = C.c_void_p()
        check(lib.sa_mlp_create(_ptr(p, C.c_float), len(p), C.byref(h)))
        self.h = h

    @staticmethod
    def n_params() -> int:
        return int(load_library().sa_mlp_n_params())

    def close(self):
        if getattr(self, "h", None):
            self._lib.sa_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params(), dtype=np.float32)
        check(self._lib.sa_mlp_get_params(self.h, _ptr(out, C.c_float), len(out)))
        return out

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], 4), dtype=torch.float32, device=X.device)
        torch.cuda.current_stream().synchronize()
        check(self._lib.sa_mlp_forward(self.h, X.shape[0], _dev(X), _dev(Y)))
        return Y

    def gradients(self, X, T):
        import torch
        g = np.empty(self.n_params(), dtype=np.float32)
        loss = C.c_double()
        torch.cuda.current_stream().synchronize()
        check(self._lib.sa_mlp_gradients(self.h, X.shape[0], _dev(X), _dev(T), _ptr(g, C.c_float), C.byref(loss)))
        return g, loss.value

    def train_step(self, X, T, lr: float) -> float:
        import torch
        loss = C.c_double()
        torch.cuda.current_stream().synchronize()
        check(self._lib.sa_mlp_train_step(self.h, X.shape[0], _dev(X), _dev(T), lr, C.byref(loss)))
        return loss.value


def from_workload(w: W.Workload, **opt_overrides) -> Model:
    return Model(w.patch, w.material, w.scan, w.options, **opt_overrides)


class MultiPatchModel:
    """Owner of one sa_multipatch handle: patches glued by the global index
    maps of their control points (workloads.glue), one or more scan paths
    (every query names its path, 0 by default)."""

    def __init__(self, patches, maps, material: W.Material, scan: W.ScanPath,
                 options: Optional[W.Options] = None, **opt_overrides):
        lib = load_library()
        self._lib = lib
        keep_list = []

        def keep(a, dtype):
            a = np.ascontiguousarray(a, dtype=dtype)
            keep_list.append(a)
            return a

        arr = (sa_patch * len(patches))()
        for i, P in enumerate(patches):
            arr[i] = _patch_struct(P, keep)
        imap = keep(np.concatenate([np.asarray(g, np.int64) for g in maps]), np.int64)
        m = sa_material(material.k, material.rho, material.cp, material.T0)
        o = _options_struct(options, opt_overrides, keep)
        s = _scan_struct(scan, o, keep)
        h = C.c_void_p()
        check(lib.sa_mp_setup(arr, len(patches), _ptr(imap, C.c_int64), C.byref(m), C.byref(s), C.byref(h)))
        self.h = h
        self.T0 = material.T0
        self.info = self.get_info()

    def close(self):
        if getattr(self, "h", None):
            self._lib.sa_mp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        check(self._lib.sa_mp_step(self.h, n))

    def get_info(self, path: int = 0) -> sa_mp_info:
        i = sa_mp_info()
        check(self._lib.sa_mp_get_info(self.h, path, C.byref(i)))
        return i

    def boundary_fields(self, path: int = 0):
        """T~ [nq], grad T~ [nq, 3] at the boundary points, F [n_dof] and
        du [n_dof] = T^ - T_c at the global control points."""
        self.info = self.get_info()
        nq, nd = self.info.n_bpts, self.info.n_dof
        T = np.empty(nq)
        G = np.empty((3, nq))
        F = np.empty(nd)
        u = np.empty(nd)
        check(self._lib.sa_mp_get_boundary_fields(self.h, path, _ptr(T, C.c_double), _ptr(G, C.c_double),
                                                  _ptr(F, C.c_double), _ptr(u, C.c_double)))
        return T, G.T.copy(), F, u

    def boundary_points(self):
        nq = self.info.n_bpts
        x = np.empty((nq, 3))
        n = np.empty((nq, 3))
        w = np.empty(nq)
        check(self._lib.sa_mp_get_boundary_points(self.h, _ptr(x, C.c_double), _ptr(n, C.c_double),
                                                  _ptr(w, C.c_double)))
        return x, n, w

    def eval_temperature(self, patch: int, xi: np.ndarray, path: int = 0):
        """T [n] and grad T [n, 3] at parametric points xi [n, 3] of one patch."""
        xi = np.ascontiguousarray(np.atleast_2d(xi), np.float64)
        n = len(xi)
        T = np.empty(n)
        G = np.empty((n, 3))
        check(self._lib.sa_mp_eval_temperature(self.h, path, patch, n, _ptr(xi, C.c_double), _ptr(T, C.c_double),
                                               _ptr(G, C.c_double)))
        return T, G

    def heat_loss(self, patch: int, face: int, edge_face: int, quad: int = 4, path: int = 0):
        """sa_mp_heat_loss: per-point x, n, ds, q~, q^ and the integrals of
        |q~ + q^| ds ("net") and |q~| ds ("tilde") along an edge of a patch."""
        n = C.c_int64(0)
        check(self._lib.sa_mp_heat_loss(self.h, path, patch, face, edge_face, quad, C.byref(n), None, None, None, None,
                                        None, None))
        m = n.value
        x, nrm, ds, qt, qh, integ = (np.empty((m, 3)), np.empty((m, 3)), np.empty(m), np.empty(m), np.empty(m),
                                     np.empty(2))
        check(self._lib.sa_mp_heat_loss(self.h, path, patch, face, edge_face, quad, C.byref(n), _ptr(x, C.c_double),
                                        _ptr(nrm, C.c_double), _ptr(ds, C.c_double), _ptr(qt, C.c_double),
                                        _ptr(qh, C.c_double), _ptr(integ, C.c_double)))
        return {"x": x, "n": nrm, "ds": ds, "q_tilde": qt, "q_hat": qh, "net": float(integ[0]),
                "tilde": float(integ[1])}

    def eval_temperature_at(self, x: np.ndarray, path: int = 0):
        """T [n], grad T [n, 3], the patch [n] (-1: in none) and the
        parametric point [n, 3] of physical points x [n, 3] (m)."""
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        n = len(x)
        T = np.empty(n)
        G = np.empty((n, 3))
        patch = np.empty(n, np.int32)
        xi = np.empty((n, 3))
        check(self._lib.sa_mp_eval_temperature_at(self.h, path, n, _ptr(x, C.c_double), _ptr(T, C.c_double),
                                                  _ptr(G, C.c_double), _ptr(patch, C.c_int32), _ptr(xi, C.c_double)))
        return T, G, patch, xi
