"""Seeded synthetic inputs: spline patches, materials and laser scan paths.

This module builds the *inputs* of the semi-analytical IGA thermal model and
nothing else.  It holds none of the model's arithmetic: no basis evaluation,
no quadrature, no kernel sum, no time stepping.  Both the FP64 CPU oracle and
the HIP library consume what it returns, so it is the one place the two sides
share.

Units are SI throughout (m, s, W, J, K).

What the inputs describe (paper, Section 2):
  * the part V as one NURBS volume patch (degree, open knot vectors, control
    net with weights), its six parametric faces tagged with their boundary
    role (Section 2, Eqs. 4-5 and 10-11: adiabatic lateral faces, Dirichlet
    bottom face, top face on the plane that holds the sources);
  * the material (k, rho, c_p, T_c) of Eqs. 1-3;
  * the discretised laser history: instantaneous point sources with position,
    integer activation tick and energy (Section 2, laser discretisation and
    the text after Eq. 8).  Source i is switched on at time tick_i * delta,
    where delta = dt / sources_per_step.

Scan paths are generated as polylines/arcs and discretised at spacing
v * delta along the path; the source activated at time (m)*delta after the
segment start sits where the laser is at that time.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Face roles (order of faces: xi0=0, xi0=1, xi1=0, xi1=1, xi2=0, xi2=1).
FACE_NEUMANN = 0        # lateral, adiabatic: receives the transferred flux load
FACE_DIRICHLET = 1      # bottom, build platform: T = T_c
FACE_SOURCE_PLANE = 2   # top: adiabatic by construction of the point-source kernel
FACE_INTERFACE = 3      # glued to a face of another patch: no boundary points, no load

PRECISION_FP64 = 0
PRECISION_FP32_FAR = 1
PRECISION_SURROGATE = 2

PRECOND_JACOBI = 0
PRECOND_FD = 1


@dataclasses.dataclass
class Patch:
    degree: Tuple[int, int, int]
    knots: Tuple[np.ndarray, np.ndarray, np.ndarray]
    ctrl: np.ndarray                    # [n2, n1, n0, 4]: x, y, z (m), weight
    face_role: Tuple[int, int, int, int, int, int]
    quad_vol: Tuple[int, int, int]
    quad_face: int = 3

    @property
    def n_ctrl(self) -> Tuple[int, int, int]:
        return (self.ctrl.shape[2], self.ctrl.shape[1], self.ctrl.shape[0])

    @property
    def n_dof(self) -> int:
        n0, n1, n2 = self.n_ctrl
        return n0 * n1 * n2

    def n_elem(self, d: int) -> int:
        return int(np.count_nonzero(np.diff(np.unique(self.knots[d])) > 0))


@dataclasses.dataclass
class Material:
    k: float        # W/(m K)
    rho: float      # kg/m^3
    cp: float       # J/(kg K)
    T0: float       # K, platform and initial temperature T_c


@dataclasses.dataclass
class ScanPath:
    """Point sources of one or more independent scan strategies (paths).

    Sources of path p occupy rows src_offset[p]:src_offset[p+1] and are sorted
    by tick (non-decreasing).  tick >= 1; n_steps[p] theta-steps of length dt
    advance path p; each step activates the next sources_per_step ticks.
    """
    src_offset: np.ndarray      # int64 [n_paths+1]
    xyz: np.ndarray             # float64 [N, 3]
    tick: np.ndarray            # int64 [N]
    energy: np.ndarray          # float64 [N] (J)
    n_steps: np.ndarray         # int32 [n_paths]
    dt: float
    sources_per_step: int
    spot_radius: float = 20e-6

    @property
    def n_paths(self) -> int:
        return len(self.n_steps)

    @property
    def delta(self) -> float:
        return self.dt / self.sources_per_step

    def path(self, p: int) -> "ScanPath":
        a, b = int(self.src_offset[p]), int(self.src_offset[p + 1])
        return ScanPath(np.array([0, b - a], np.int64), self.xyz[a:b].copy(),
                        self.tick[a:b].copy(), self.energy[a:b].copy(),
                        self.n_steps[p:p + 1].copy(), self.dt,
                        self.sources_per_step, self.spot_radius)


@dataclasses.dataclass
class Options:
    theta: float = 0.5
    kernel_scale: float = 1.0
    precision: int = PRECISION_FP64
    tau_near: float = 2e-4
    pcg_rtol: float = 1e-13
    pcg_max_iter: int = 2000
    preconditioner: int = PRECOND_FD


@dataclasses.dataclass
class Workload:
    name: str
    patch: Patch
    material: Material
    scan: ScanPath
    options: Options


# ----------------------------------------------------------------------------
# knot vectors and control nets
# ----------------------------------------------------------------------------

def open_uniform_knots(n_el: int, p: int) -> np.ndarray:
    inner = [i / n_el for i in range(1, n_el)]
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1))


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae: control parameters that make a B-spline curve with
    control values g(xi*_a) reproduce any affine function g exactly."""
    n = len(knots) - p - 1
    if p == 0:
        return 0.5 * (knots[:n] + knots[1:n + 1])
    return np.array([knots[a + 1:a + p + 1].mean() for a in range(n)])


def insert_knot_curve(knots, p, Pw, u):
    """Boehm knot insertion on a curve in homogeneous coordinates.

    Pw: [n, dim] homogeneous control points (w*x, ..., w).  Returns the new
    knot vector and control points; the curve is unchanged."""
    knots = np.asarray(knots, float)
    n = Pw.shape[0]
    k = int(np.searchsorted(knots, u, side="right") - 1)
    k = min(k, len(knots) - p - 2)
    Q = np.empty((n + 1, Pw.shape[1]))
    Q[:k - p + 1] = Pw[:k - p + 1]
    Q[k + 1:] = Pw[k:]
    for i in range(k - p + 1, k + 1):
        den = knots[i + p] - knots[i]
        a = 0.0 if den == 0 else (u - knots[i]) / den
        Q[i] = a * Pw[i] + (1.0 - a) * Pw[i - 1]
    new_knots = np.concatenate([knots[:k + 1], [u], knots[k + 1:]])
    return new_knots, Q


def refine_curve(knots, p, Pw, new_knots: Sequence[float]):
    for u in new_knots:
        knots, Pw = insert_knot_curve(knots, p, Pw, u)
    return knots, Pw


def block_patch(lo, hi, n_el, degree, roles=None, quad_vol=None, quad_face=3) -> Patch:
    """Axis-aligned box [lo, hi] as a B-spline volume (unit weights, control
    points at Greville abscissae, so the map is affine)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    if np.isscalar(degree):
        degree = (degree,) * 3
    knots = tuple(open_uniform_knots(n_el[d], degree[d]) for d in range(3))
    g = [lo[d] + (hi[d] - lo[d]) * greville(knots[d], degree[d]) for d in range(3)]
    X2, X1, X0 = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    ctrl = np.stack([X0, X1, X2, np.ones_like(X0)], axis=-1)
    if roles is None:
        roles = (FACE_NEUMANN,) * 4 + (FACE_DIRICHLET, FACE_SOURCE_PLANE)
    if quad_vol is None:
        quad_vol = tuple(d + 1 for d in degree)
    return Patch(tuple(degree), knots, ctrl, tuple(roles), tuple(quad_vol), quad_face)


def annulus_patch(r_in, r_out, height, n_el=(48, 24, 12), degree=2, roles=None,
                  quad_vol=None, quad_face=3) -> Patch:
    """Quarter annulus (angle 0..pi/2 about the z axis) extruded along z.

    xi0 = angle (rational quadratic arc with the exact circular weights,
    refined by knot insertion), xi1 = radius, xi2 = height.  The angular
    direction is always quadratic (exact circle); the other two use `degree`.
    """
    p0 = 2
    k0 = np.array([0, 0, 0, 1, 1, 1], float)
    w_mid = math.sqrt(0.5)
    Pw = np.array([[1.0, 0.0, 1.0], [w_mid, w_mid, w_mid], [0.0, 1.0, 1.0]])
    k0, Pw = refine_curve(k0, p0, Pw, [i / n_el[0] for i in range(1, n_el[0])])
    wa = Pw[:, 2]
    ca = Pw[:, :2] / wa[:, None]
    p1 = p2 = degree
    k1 = open_uniform_knots(n_el[1], p1)
    k2 = open_uniform_knots(n_el[2], p2)
    r = r_in + (r_out - r_in) * greville(k1, p1)
    z = height * greville(k2, p2)
    n0, n1, n2 = len(wa), len(r), len(z)
    ctrl = np.empty((n2, n1, n0, 4))
    for a2 in range(n2):
        for a1 in range(n1):
            ctrl[a2, a1, :, 0] = r[a1] * ca[:, 0]
            ctrl[a2, a1, :, 1] = r[a1] * ca[:, 1]
            ctrl[a2, a1, :, 2] = z[a2]
            ctrl[a2, a1, :, 3] = wa
    if roles is None:
        roles = (FACE_NEUMANN,) * 4 + (FACE_DIRICHLET, FACE_SOURCE_PLANE)
    deg = (p0, p1, p2)
    if quad_vol is None:
        quad_vol = tuple(d + 1 for d in deg)
    return Patch(deg, (k0, k1, k2), ctrl, tuple(roles), tuple(quad_vol), quad_face)


# The cube with a quarter cylinder removed (paper, Section 3.1, Table 2 and the
# knot vectors printed with it).  Table 2 lists the top-surface net in mm.  The
# weights are not printed; the arc control points lie on a circle of radius
# 1 mm about (2, 0), so the middle points carry cos(pi/8) (exact circle).
E1_TOP_NET_MM = np.array([
    [[1.0, 0.0, 2.0], [0.0, 0.0, 2.0]],
    [[1.0, math.sqrt(2.0) - 1.0, 2.0], [0.0, 1.0, 2.0]],
    [[2.0 - math.sqrt(2.0) / 2.0, math.sqrt(2.0) / 2.0, 2.0], [0.0, 2.0, 2.0]],
    [[3.0 - math.sqrt(2.0), 1.0, 2.0], [1.0, 2.0, 2.0]],
    [[2.0, 1.0, 2.0], [2.0, 2.0, 2.0]],
])
E1_KNOTS = (np.array([0, 0, 0, 0.5, 0.5, 1, 1, 1], float),
            np.array([0, 0, 1, 1], float), np.array([0, 0, 1, 1], float))


def e1_patch(top_net_mm: Optional[np.ndarray] = None, roles=None) -> Patch:
    """Coarse NURBS patch of the Section 3.1 part (unrefined, as printed)."""
    net = E1_TOP_NET_MM if top_net_mm is None else np.asarray(top_net_mm, float)
    w_mid = math.cos(math.pi / 8.0)
    wts = np.array([1.0, w_mid, 1.0, w_mid, 1.0])
    ctrl = np.empty((2, 2, 5, 4))
    for a2, zmm in enumerate((0.0, 2.0)):
        for a1 in range(2):
            for a0 in range(5):
                ctrl[a2, a1, a0, :2] = net[a0, a1, :2] * 1e-3
                ctrl[a2, a1, a0, 2] = zmm * 1e-3
                ctrl[a2, a1, a0, 3] = wts[a0]
    if roles is None:
        roles = (FACE_NEUMANN,) * 4 + (FACE_DIRICHLET, FACE_SOURCE_PLANE)
    return Patch((2, 1, 1), E1_KNOTS, ctrl, tuple(roles), (3, 2, 2), 3)


def _along_axis(ctrl, d, fn):
    """Apply fn(Pw [n, 4]) -> Pw' [n', 4] to every row of homogeneous control
    points along parametric axis d of ctrl [n2][n1][n0][4] (x, y, z, w)."""
    ax = 2 - d                                       # array axis of parametric direction d
    Pw = np.concatenate([ctrl[..., :3] * ctrl[..., 3:], ctrl[..., 3:]], axis=-1)
    moved = np.moveaxis(Pw, ax, -2)                  # [..., n_d, 4]
    rows = moved.reshape(-1, moved.shape[-2], 4)
    out = np.stack([fn(r) for r in rows])
    out = out.reshape(moved.shape[:-2] + out.shape[-2:])
    out = np.moveaxis(out, -2, ax)
    return np.concatenate([out[..., :3] / out[..., 3:], out[..., 3:]], axis=-1)


def refine_patch(patch: Patch, splits: Sequence[int], degree: int = 2) -> Patch:
    """h-refinement of a patch: directions of degree 1 with a single element
    are first raised to `degree` 2 (a linear Bezier segment P0, P1 becomes
    P0, (P0 + P1)/2, P1 in homogeneous coordinates), then every element of
    direction d is cut into splits[d] equal parametric parts by knot
    insertion; the geometry map is unchanged and existing interior knots
    keep their multiplicity (so a C0 line stays C0)."""
    ctrl = np.array(patch.ctrl, float)
    knots = [np.asarray(k, float) for k in patch.knots]
    deg = list(patch.degree)
    for d in range(3):
        if deg[d] == 1 and degree == 2:
            if len(knots[d]) != 4:
                raise ValueError("degree elevation is written for a single linear element")
            ctrl = _along_axis(ctrl, d, lambda r: np.stack([r[0], 0.5 * (r[0] + r[1]), r[1]]))
            knots[d] = np.array([knots[d][0]] * 3 + [knots[d][-1]] * 3)
            deg[d] = 2
        new = []
        t = knots[d]
        for lo, hi in zip(t[:-1], t[1:]):
            if hi > lo:
                new.extend(lo + (hi - lo) * np.arange(1, splits[d]) / splits[d])
        if new:
            k0 = knots[d]
            ctrl = _along_axis(ctrl, d, lambda r, k0=k0, p=deg[d]: refine_curve(k0, p, r, new)[1])
            knots[d] = refine_curve(k0, deg[d], np.zeros((len(k0) - deg[d] - 1, 4)), new)[0]
    return Patch(tuple(deg), tuple(knots), ctrl, patch.face_role, tuple(max(q, deg[i] + 1) for i, q in
                                                                        enumerate(patch.quad_vol)), patch.quad_face)


# ----------------------------------------------------------------------------
# scan paths -> point sources
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Segment:
    kind: str            # "line" or "arc"
    power: float         # absorbed power (W)
    speed: float         # m/s
    p0: np.ndarray = None
    p1: np.ndarray = None
    center: np.ndarray = None
    radius: float = 0.0
    ang0: float = 0.0
    ang1: float = 0.0
    z: float = 0.0

    def length(self) -> float:
        if self.kind == "line":
            return float(np.linalg.norm(np.asarray(self.p1) - np.asarray(self.p0)))
        return abs(self.ang1 - self.ang0) * self.radius

    def at(self, s: np.ndarray) -> np.ndarray:
        if self.kind == "line":
            p0 = np.asarray(self.p0, float)
            d = (np.asarray(self.p1, float) - p0) / self.length()
            return p0[None, :] + s[:, None] * d[None, :]
        sgn = 1.0 if self.ang1 >= self.ang0 else -1.0
        ang = self.ang0 + sgn * s / self.radius
        c = np.asarray(self.center, float)
        return np.stack([c[0] + self.radius * np.cos(ang),
                         c[1] + self.radius * np.sin(ang),
                         np.full_like(ang, self.z)], axis=1)


def sources_from_segments(segments: List[Segment], delta: float, tick0: int = 0,
                          max_sources: Optional[int] = None):
    """Discretise segments into point sources: source m (m = 1, 2, ...) of a
    segment sits at arc length m*v*delta from its start; ticks run on across
    segments with no jump time.  Segments shorter than one spacing give none."""
    xyz, tick, energy = [], [], []
    t = tick0
    for seg in segments:
        spacing = seg.speed * delta
        m = int(math.floor(seg.length() / spacing + 1e-9))
        if m <= 0:
            continue
        s = spacing * np.arange(1, m + 1)
        xyz.append(seg.at(s))
        tick.append(t + np.arange(1, m + 1, dtype=np.int64))
        energy.append(np.full(m, seg.power * delta))
        t += m
    if not xyz:
        return np.zeros((0, 3)), np.zeros(0, np.int64), np.zeros(0)
    xyz = np.concatenate(xyz)
    tick = np.concatenate(tick)
    energy = np.concatenate(energy)
    if max_sources is not None:
        xyz, tick, energy = xyz[:max_sources], tick[:max_sources], energy[:max_sources]
    return xyz, tick, energy


def make_scan(paths, dt, n_s, spot_radius=20e-6, n_steps=None) -> ScanPath:
    """paths: list of (xyz, tick, energy) per path."""
    off = [0]
    for p in paths:
        off.append(off[-1] + len(p[1]))
    xyz = np.concatenate([p[0] for p in paths]) if off[-1] else np.zeros((0, 3))
    tick = np.concatenate([p[1] for p in paths]).astype(np.int64) if off[-1] else np.zeros(0, np.int64)
    en = np.concatenate([p[2] for p in paths]) if off[-1] else np.zeros(0)
    if n_steps is None:
        n_steps = [int(math.ceil(int(p[1][-1]) / n_s)) if len(p[1]) else 0 for p in paths]
    return ScanPath(np.array(off, np.int64), np.ascontiguousarray(xyz, float),
                    np.ascontiguousarray(tick), np.ascontiguousarray(en, float),
                    np.array(n_steps, np.int32), float(dt), int(n_s), float(spot_radius))


def hatch_rect_segments(x0, x1, y0, y1, z, angle_deg, hatch, power, speed, rng=None,
                        jitter=0.0):
    """Boustrophedon hatch lines at angle_deg over the rectangle, spacing
    `hatch`, each start moved inward by U[0, jitter] along the line."""
    a = math.radians(angle_deg)
    d = np.array([math.cos(a), math.sin(a)])
    nrm = np.array([-math.sin(a), math.cos(a)])
    corners = np.array([[x0, y0], [x1, y0], [x0, y1], [x1, y1]])
    c = corners @ nrm
    cmin, cmax = c.min(), c.max()
    segs = []
    k = 0
    while True:
        off = cmin + (k + 0.5) * hatch
        if off >= cmax:
            break
        base = off * nrm
        # clip the line base + s d to the rectangle
        lo, hi = -np.inf, np.inf
        ok = True
        for dim, (bmin, bmax) in enumerate(((x0, x1), (y0, y1))):
            if abs(d[dim]) < 1e-15:
                if not (bmin <= base[dim] <= bmax):
                    ok = False
                continue
            s_a = (bmin - base[dim]) / d[dim]
            s_b = (bmax - base[dim]) / d[dim]
            lo = max(lo, min(s_a, s_b))
            hi = min(hi, max(s_a, s_b))
        if ok and hi > lo:
            if k % 2 == 1:
                lo, hi = hi, lo
            j = rng.uniform(0.0, jitter) if (rng is not None and jitter > 0) else 0.0
            sgn = 1.0 if hi > lo else -1.0
            lo = lo + sgn * j
            p0 = np.array([*(base + lo * d), z])
            p1 = np.array([*(base + hi * d), z])
            if (hi - lo) * sgn > 0:
                segs.append(Segment("line", power, speed, p0=p0, p1=p1))
        k += 1
    return segs


# ----------------------------------------------------------------------------
# workloads (sizes of the five benchmark configurations)
# ----------------------------------------------------------------------------

MAT_CFG = Material(k=20.0, rho=4430.0, cp=560.0, T0=293.0)
MAT_TI64 = Material(k=42.0, rho=4420.0, cp=990.0, T0=293.0)   # paper Table 1


def cfg1(options: Optional[Options] = None) -> Workload:
    """Block 2x1x1 mm, quadratic B-splines 16x8x8, one straight 1.5 mm track
    at y = 0.5 mm on the top face, 40 W absorbed, 1 m/s, dt = 10 us, 10
    sources per step (150 steps, 1500 sources), theta = 0.5."""
    patch = block_patch((0, 0, 0), (2e-3, 1e-3, 1e-3), (16, 8, 8), 2)
    seg = Segment("line", 40.0, 1.0, p0=np.array([0.25e-3, 0.5e-3, 1e-3]),
                  p1=np.array([1.75e-3, 0.5e-3, 1e-3]))
    dt, n_s = 1e-5, 10
    src = sources_from_segments([seg], dt / n_s)
    scan = make_scan([src], dt, n_s)
    return Workload("cfg1_block_track_p2", patch, MAT_CFG, scan, options or Options())


def raster_segments(seed: int, n_tracks=10, y0=0.55e-3, hatch=0.1e-3, x0=0.1e-3,
                    x1=3.9e-3, z=1e-3, power=80.0, speed=1.0, jitter=20e-6):
    rng = np.random.Generator(np.random.PCG64(seed))
    segs = []
    for k in range(n_tracks):
        j = rng.uniform(0.0, jitter)
        y = y0 + k * hatch
        if k % 2 == 0:
            p0, p1 = (x0 + j, y, z), (x1, y, z)
        else:
            p0, p1 = (x1 - j, y, z), (x0, y, z)
        segs.append(Segment("line", power, speed, p0=np.array(p0), p1=np.array(p1)))
    return segs


def cfg2(seed: int = 0, options: Optional[Options] = None, n_el=(64, 32, 16), degree=3,
         n_tracks=10) -> Workload:
    """Block 4x2x1 mm, cubic B-splines 64x32x16; 10 boustrophedon tracks
    along x (0.1 mm hatch, 0.1 mm border, start jitter U[0,20] um), 80 W,
    1 m/s, dt = 10 us, 5 sources per step (about 3,800 steps, 19k sources)."""
    patch = block_patch((0, 0, 0), (4e-3, 2e-3, 1e-3), n_el, degree)
    dt, n_s = 1e-5, 5
    src = sources_from_segments(raster_segments(seed, n_tracks=n_tracks), dt / n_s)
    scan = make_scan([src], dt, n_s)
    return Workload("cfg2_block_raster_p3", patch, MAT_CFG, scan, options or Options())


def annulus_scan_segments(seed: int, r_c=3.5e-3, r_in=2e-3, hatch=0.1e-3, z=1e-3,
                          speed=0.8, p_lo=60.0, p_hi=100.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    segs = [Segment("arc", rng.uniform(p_lo, p_hi), speed, center=np.zeros(2),
                    radius=r_c, ang0=0.0, ang1=math.pi / 2, z=z)]
    nrm = np.array([1.0, -1.0]) / math.sqrt(2.0)
    tan = np.array([1.0, 1.0]) / math.sqrt(2.0)
    dmax = r_c / math.sqrt(2.0)
    n_lines = int(math.floor(dmax / hatch + 1e-9))
    k = 0
    for i in range(-n_lines, n_lines + 1):
        dd = i * hatch
        s_lo = abs(dd)
        if abs(dd) < r_in:
            s_lo = max(s_lo, math.sqrt(r_in * r_in - dd * dd))
        s_hi2 = r_c * r_c - dd * dd
        if s_hi2 <= 0:
            continue
        s_hi = math.sqrt(s_hi2)
        if s_hi <= s_lo:
            continue
        a, b = (s_lo, s_hi) if k % 2 == 0 else (s_hi, s_lo)
        p0 = np.array([*(dd * nrm + a * tan), z])
        p1 = np.array([*(dd * nrm + b * tan), z])
        segs.append(Segment("line", rng.uniform(p_lo, p_hi), speed, p0=p0, p1=p1))
        k += 1
    return segs


def cfg3(seed: int = 0, options: Optional[Options] = None, n_el=(48, 24, 12)) -> Workload:
    """Quarter annulus r in [2, 4] mm, 1 mm tall, quadratic NURBS 48x24x12;
    contour pass at r = 3.5 mm then 45-degree hatches (0.1 mm) clipped to the
    contour, P ~ U[60, 100] W per track, 0.8 m/s, 8 sources per step."""
    patch = annulus_patch(2e-3, 4e-3, 1e-3, n_el, 2)
    dt, n_s = 1e-5, 8
    src = sources_from_segments(annulus_scan_segments(seed), dt / n_s)
    scan = make_scan([src], dt, n_s)
    opts = options or Options(precision=PRECISION_FP32_FAR)
    return Workload("cfg3_annulus_contour_hatch_p2", patch, MAT_CFG, scan, opts)


ANGLES_CFG4 = (0.0, 45.0, 67.0, 90.0)


def strategy_segments(rng, lx=4e-3, ly=2e-3, z=1e-3, border=0.1e-3, hatch=0.1e-3):
    ang = float(rng.choice(ANGLES_CFG4))
    L = int(rng.integers(500, 4001))
    P = float(rng.uniform(40.0, 120.0))
    v = float(rng.uniform(0.6, 1.5))
    segs = hatch_rect_segments(border, lx - border, border, ly - border, z, ang, hatch,
                               P, v, rng=rng, jitter=20e-6)
    return segs, L, ang, P, v


def cfg4(seed: int = 0, n_strategies: int = 128, options: Optional[Options] = None,
         n_el=(64, 32, 16), degree=3, max_len: Optional[int] = None) -> Workload:
    """n_strategies independent scan strategies on the cfg2 block, each of
    U[500, 4000] steps, hatch angle from {0, 45, 67, 90} deg, absorbed power
    U[40, 120] W, speed U[0.6, 1.5] m/s (drawn in that order per strategy)."""
    patch = block_patch((0, 0, 0), (4e-3, 2e-3, 1e-3), n_el, degree)
    dt, n_s = 1e-5, 5
    rng = np.random.Generator(np.random.PCG64(seed))
    paths, steps = [], []
    for _ in range(n_strategies):
        segs, L, _, _, _ = strategy_segments(rng)
        if max_len is not None:
            L = min(L, max_len)
        src = sources_from_segments(segs, dt / n_s, max_sources=L * n_s)
        paths.append(src)
        steps.append(L)
    scan = make_scan(paths, dt, n_s, n_steps=steps)
    opts = options or Options(precision=PRECISION_FP32_FAR)
    return Workload("cfg4_block_batch128", patch, MAT_CFG, scan, opts)


def small_block(n_el=(4, 3, 3), degree=2, size=(1e-3, 0.6e-3, 0.5e-3), roles=None) -> Patch:
    return block_patch((0, 0, 0), size, n_el, degree, roles=roles)


def single_track(p0, p1, power, speed, dt, n_s, spot_radius=20e-6) -> ScanPath:
    seg = Segment("line", power, speed, p0=np.asarray(p0, float), p1=np.asarray(p1, float))
    src = sources_from_segments([seg], dt / n_s)
    return make_scan([src], dt, n_s, spot_radius=spot_radius)


# Section 3.1 and 3.2 experiments on the part of Table 2 (2 mm cube without a
# quarter cylinder of radius 1 mm about (2, 0) mm): Ti-6Al-4V (Table 1),
# P = 82.5 W, A = 0.77, one source per dt = 10 us, r = 20 um.  The printed
# heat-loss integrals of these experiments (Tables 3-4) are matched by the
# kernel with the half-space factor s = 2, which these workloads use.
MAT_TI64 = Material(k=42.0, rho=4420.0, cp=990.0, T0=293.0)
E_PAPER = 0.77 * 82.5 * 1e-5


def e1(splits=(8, 10, 20), options: Optional[Options] = None) -> Workload:
    """Single source (Sec. 3.1): 100 um from the arc on its 45-degree line,
    on the top face, switched on in the first step; after 20 steps its age
    is 1.9e-4 s, the comparison time of the paper.  splits cut the elements
    of the Table 2 patch (raised to quadratic) along (arc, radius, height)."""
    patch = refine_patch(e1_patch(), splits)
    d = 1.1e-3 / math.sqrt(2.0)
    src = (np.array([[2e-3 - d, d, 2e-3]]), np.array([1], np.int64), np.array([E_PAPER]))
    scan = make_scan([src], 1e-5, 1, n_steps=[20])
    return Workload("e1_single_source", patch, MAT_TI64, scan, options or Options(kernel_scale=2.0))


def e2(splits=(8, 10, 20), options: Optional[Options] = None) -> Workload:
    """Contour scan (Sec. 3.2): 0.5 m/s along the arc at 100 um from the
    curved face (radius 1.1 mm about (2, 0) mm), from the face y = 0 to the
    face x = 2 mm, one source per 10 us (5 um apart), 345 steps."""
    patch = refine_patch(e1_patch(), splits)
    seg = Segment("arc", 0.77 * 82.5, 0.5, center=np.array([2e-3, 0.0]), radius=1.1e-3, ang0=math.pi,
                  ang1=math.pi / 2, z=2e-3)
    scan = make_scan([sources_from_segments([seg], 1e-5)], 1e-5, 1)
    return Workload("e2_contour_scan", patch, MAT_TI64, scan, options or Options(kernel_scale=2.0))


# ----------------------------------------------------------------------------
# several patches glued conformingly (multi-patch parts)
# ----------------------------------------------------------------------------

def block_patch_knots(lo, hi, knots, degree, roles, quad_vol=None, quad_face=3) -> Patch:
    """Axis-aligned box [lo, hi] on the given knot vectors (control points at
    their Greville abscissae, so the map is affine)."""
    lo = np.asarray(lo, float)
    hi = np.asarray(hi, float)
    if np.isscalar(degree):
        degree = (degree,) * 3
    knots = tuple(np.asarray(k, float) for k in knots)
    g = [lo[d] + (hi[d] - lo[d]) * greville(knots[d], degree[d]) for d in range(3)]
    X2, X1, X0 = np.meshgrid(g[2], g[1], g[0], indexing="ij")
    ctrl = np.stack([X0, X1, X2, np.ones_like(X0)], axis=-1)
    if quad_vol is None:
        quad_vol = tuple(d + 1 for d in degree)
    return Patch(tuple(degree), knots, ctrl, tuple(roles), tuple(quad_vol), quad_face)


def glue(patches, rel_tol=1e-9):
    """Global numbering of the control points of patches that meet face to
    face with matching control points: points of different patches at the
    same position (within rel_tol of the part's extent) share one index.
    Returns the index map of each patch (control point order of the patch)
    and the number of global control points.  Shared points must carry the
    same weight."""
    P = np.concatenate([p.ctrl.reshape(-1, 4) for p in patches])
    ext = float(np.abs(P[:, :3] - P[:, :3].mean(axis=0)).max())
    key = np.round(P[:, :3] / (rel_tol * ext)).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    if not np.allclose(P[:, 3], P[first[inv], 3], rtol=1e-12, atol=0.0):
        raise ValueError("shared control points carry different weights")
    # global indices in order of first appearance
    order = np.argsort(first)
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    g = rank[inv]
    maps, o = [], 0
    for p in patches:
        maps.append(g[o:o + p.n_dof].astype(np.int64))
        o += p.n_dof
    return maps, int(len(first))


@dataclasses.dataclass
class MultiWorkload:
    name: str
    patches: List[Patch]
    maps: List[np.ndarray]
    material: Material
    scan: ScanPath
    options: Options


def l_part(n_el=(8, 8, 4), degree=2, size=(1e-3, 1e-3, 0.5e-3), power=80.0, speed=1.0,
           options: Optional[Options] = None) -> MultiWorkload:
    """L-shaped plan from three conforming patches: the corner square
    [0, a]^2 and the arms [a, a+b] x [0, a] and [0, a] x [a, a+b], height h
    (size = (a, b, h)); n_el = elements along a, along b and along h.  The
    faces where the patches meet are interfaces; bottom Dirichlet, top
    source plane, the outer sides adiabatic.  One track along the L's centre
    line, from the end of the x arm through the corner to the end of the y
    arm (0.2 mm from the ends), 10 us steps, 5 sources per step."""
    a, b, h = size
    na, nb, nz = n_el
    ka, kb, kz = (open_uniform_knots(n, degree) for n in (na, nb, nz))
    N, D, S, I = FACE_NEUMANN, FACE_DIRICHLET, FACE_SOURCE_PLANE, FACE_INTERFACE
    corner = block_patch_knots((0, 0, 0), (a, a, h), (ka, ka, kz), degree, (N, I, N, I, D, S))
    arm_x = block_patch_knots((a, 0, 0), (a + b, a, h), (kb, ka, kz), degree, (I, N, N, N, D, S))
    arm_y = block_patch_knots((0, a, 0), (a, a + b, h), (ka, kb, kz), degree, (N, N, I, N, D, S))
    patches = [corner, arm_x, arm_y]
    maps, _ = glue(patches)
    c = 0.5 * a
    segs = [Segment("line", power, speed, p0=np.array([a + b - 0.2e-3, c, h]), p1=np.array([c, c, h])),
            Segment("line", power, speed, p0=np.array([c, c, h]), p1=np.array([c, a + b - 0.2e-3, h]))]
    dt, n_s = 1e-5, 5
    scan = make_scan([sources_from_segments(segs, dt / n_s)], dt, n_s)
    return MultiWorkload("l_part_three_patches", patches, maps, MAT_CFG, scan, options or Options())


WORKLOADS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4, "e1": e1, "e2": e2}
