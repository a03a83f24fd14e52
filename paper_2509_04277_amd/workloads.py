"""Seeded synthetic rod workloads: plain data shared by the tests, the benchmark and the oracle.

This module holds input *descriptions* only: geometry, material constants, clamp motion and
initial states drawn from seeded numpy generators.  It contains none of the stepping method's
arithmetic (no stiffness, mass, inertia, force, constraint or integration formula); both the
GPU library and the CPU oracle derive those from the raw material description on their own.

Workloads (free-space tests of Sec. 3.1 and the two-instrument set-up of Sec. 3.4, without
the anatomy meshes, which are not available):
  c0  one extensible rod, 64 elements, 1 m, r = 1 cm, E = 1 MPa, nu = 0.5, rho = 1000,
      clamped at the origin pointing along +x, Gaussian lateral noise sigma = 1 mm on the
      free points, frames aligned to the segments, 2000 steps at half the largest stable dt.
  c1  two inextensible rods of 512 elements (1 m each), rod A r = 0.5 mm, E = 2 GPa; rod B
      r = 0.2 mm, E = 50 GPa with the last 26 elements at 5 GPa, 5 mm apart, no contact, each
      base driven by a seeded sinusoidal insertion (amplitude l/20) and twist (0.2 rad) making
      two periods over 20000 steps; 10 constraint iterations.  (An insertion amplitude of
      l/2 at this frequency buckles rod A dynamically and makes the trajectory chaotic.)
  c2  single long rod, N in {1024, 4096, 16384, 65536}, element length 1/64 m, c0 material,
      seeded Gaussian initial curvature sigma = 0.05 rad per element.
  c3  4096 rods, N log-uniform in [32, 2048], E log-uniform in [1e6, 1e10] Pa, r uniform in
      [0.1, 1] mm, element length 1/64 m, half extensible / half inextensible, each with its
      own dt (left 0 here: set from the stability rule by the caller).
  c4  256 rods x 256 elements, inextensible, c0 material, L = 4 m, curvature and twist noise,
      dt from the stability rule (left 0 here), 400 steps, checkpoints every 20 steps.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DT_GOLDEN = os.path.join(REPO, "tests", "golden", "dt_bisect.json")


@dataclass
class RodSpec:
    """Raw description of one rod (SI units)."""
    n: int
    inextensible: bool
    n_iter: int
    clamp: bool
    dt: float
    gravity: Tuple[float, float, float]
    damp_lin: float
    damp_ang: float
    poisson: float
    density: float
    seg_len: np.ndarray
    radius: np.ndarray
    young: np.ndarray
    kp_scale: float = 1.0
    bend_scale: float = 1.0
    twist_scale: float = 1.0
    u_hat: Optional[np.ndarray] = None
    f_ext: Optional[np.ndarray] = None
    tau_ext: Optional[np.ndarray] = None
    clamp_x0: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    clamp_q0: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)
    clamp_amp: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    clamp_twist_amp: float = 0.0
    clamp_twist_axis: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    clamp_freq: float = 0.0
    clamp_phase_x: float = 0.0
    clamp_phase_twist: float = 0.0
    damp_int: float = 0.0   # internal friction: Kelvin-Voigt retardation time [s]

    def replace(self, **kw) -> "RodSpec":
        return dataclasses.replace(self, **kw)


@dataclass
class RodState:
    """Rod state: x, v (N+1, 3); q (N, 4) as (w, x, y, z); w = body angular velocity (N, 3)."""
    x: np.ndarray
    v: np.ndarray
    q: np.ndarray
    w: np.ndarray

    def copy(self) -> "RodState":
        return RodState(self.x.copy(), self.v.copy(), self.q.copy(), self.w.copy())

    def astype(self, dt) -> "RodState":
        return RodState(*(np.ascontiguousarray(a, dtype=dt) for a in (self.x, self.v, self.q, self.w)))


@dataclass
class Workload:
    name: str
    rods: List[Tuple[RodSpec, RodState]]
    n_steps: int
    steps_per_launch: int
    meta: dict = field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return sum(s.n for s, _ in self.rods)


# ----------------------------------------------------------------- initial geometry --
# Quaternion helpers used only to *construct* initial frames (input preparation).

def _qprod(a, b):
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _min_rotation(a, b):
    """Unit quaternion of the smallest rotation taking unit vector a to unit vector b."""
    c = np.cross(a, b)
    q = np.array([1.0 + float(np.dot(a, b)), c[0], c[1], c[2]])
    return q / np.linalg.norm(q)


def _third_axis(q):
    w, x, y, z = q
    return np.array([2 * (x * z + w * y), 2 * (y * z - w * x), w * w - x * x - y * y + z * z])


def _axis_angle(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    nrm = np.linalg.norm(axis)
    if nrm == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    s = math.sin(0.5 * angle) / nrm
    return np.array([math.cos(0.5 * angle), axis[0] * s, axis[1] * s, axis[2] * s])


Q_ALONG_X = np.array([math.cos(math.pi / 4), 0.0, math.sin(math.pi / 4), 0.0])  # e3 -> +x


def frames_from_polyline(x: np.ndarray) -> np.ndarray:
    """Frames aligned to the segments of polyline x by parallel transport (zero twist)."""
    n = x.shape[0] - 1
    t = x[1:] - x[:-1]
    t = t / np.linalg.norm(t, axis=1, keepdims=True)
    q = np.zeros((n, 4))
    q[0] = _min_rotation(np.array([0.0, 0.0, 1.0]), t[0])
    for j in range(n - 1):
        q[j + 1] = _qprod(_min_rotation(t[j], t[j + 1]), q[j])
        q[j + 1] /= np.linalg.norm(q[j + 1])
    return q


def curved_rod(n: int, l: float, rng, sigma: float, twist_sigma: float = 0.0,
               q0=Q_ALONG_X, x0=(0.0, 0.0, 0.0)):
    """Polyline grown from a base frame by seeded body-axis rotations per element."""
    th = rng.normal(0.0, sigma, size=(n, 3))
    th[:, 2] = rng.normal(0.0, twist_sigma, size=n) if twist_sigma > 0 else 0.0
    q = np.zeros((n, 4))
    x = np.zeros((n + 1, 3))
    q[0] = np.asarray(q0, dtype=np.float64)
    x[0] = x0
    for j in range(n):
        x[j + 1] = x[j] + l * _third_axis(q[j])
        if j + 1 < n:
            a = th[j]
            q[j + 1] = _qprod(q[j], _axis_angle(a, float(np.linalg.norm(a))))
            q[j + 1] /= np.linalg.norm(q[j + 1])
    return x, q


def curved_rods(ns, l: float, rng, sigma: float, twist_sigma: float = 0.0, q0=Q_ALONG_X):
    """Many curved rods at once (same construction as ``curved_rod``, vectorised over rods).

    Per rod, in order: body-axis angles theta ~ N(0, sigma^2) for axes 1-2 (and N(0,
    twist_sigma^2) for axis 3), one triple per element; rods of similar length are grown
    together."""
    ns = [int(n) for n in ns]
    angles = []
    for n in ns:
        th = np.zeros((n, 3))
        th[:, :2] = rng.normal(0.0, sigma, size=(n, 2))
        if twist_sigma > 0:
            th[:, 2] = rng.normal(0.0, twist_sigma, size=n)
        angles.append(th)
    out = [None] * len(ns)
    order = np.argsort(ns, kind="stable")
    for k in range(0, len(ns), 256):
        idx = order[k:k + 256]
        res = _grow_rods([angles[i] for i in idx], l, q0)
        for i, rq in zip(idx, res):
            out[i] = rq
    return out


def _grow_rods(angles, l, q0):
    ns = [a.shape[0] for a in angles]
    R, nmax = len(ns), max(ns)
    th = np.zeros((R, nmax, 3))
    for r, a in enumerate(angles):
        th[r, :a.shape[0]] = a
    th = np.ascontiguousarray(th.transpose(1, 0, 2))          # element-major: (nmax, R, 3)
    ang = np.linalg.norm(th, axis=2)
    safe = np.where(ang > 0, ang, 1.0)
    rot = np.concatenate([np.cos(0.5 * ang)[..., None],
                          (np.sin(0.5 * ang) / safe)[..., None] * th], axis=2)
    q = np.zeros((nmax, R, 4))
    x = np.zeros((nmax + 1, R, 3))
    q[0] = np.asarray(q0, dtype=np.float64)
    for j in range(nmax):
        w_, x_, y_, z_ = q[j, :, 0], q[j, :, 1], q[j, :, 2], q[j, :, 3]
        x[j + 1, :, 0] = x[j, :, 0] + l * (2 * (x_ * z_ + w_ * y_))
        x[j + 1, :, 1] = x[j, :, 1] + l * (2 * (y_ * z_ - w_ * x_))
        x[j + 1, :, 2] = x[j, :, 2] + l * (w_ * w_ - x_ * x_ - y_ * y_ + z_ * z_)
        if j + 1 < nmax:
            bw, bx, by, bz = rot[j, :, 0], rot[j, :, 1], rot[j, :, 2], rot[j, :, 3]
            nw = w_ * bw - x_ * bx - y_ * by - z_ * bz
            nx = w_ * bx + x_ * bw + y_ * bz - z_ * by
            ny = w_ * by - x_ * bz + y_ * bw + z_ * bx
            nz = w_ * bz + x_ * by - y_ * bx + z_ * bw
            inv = 1.0 / np.sqrt(nw * nw + nx * nx + ny * ny + nz * nz)
            q[j + 1, :, 0] = nw * inv
            q[j + 1, :, 1] = nx * inv
            q[j + 1, :, 2] = ny * inv
            q[j + 1, :, 3] = nz * inv
    x = x.transpose(1, 0, 2)
    q = q.transpose(1, 0, 2)
    return [(x[r, :n + 1].copy(), q[r, :n].copy()) for r, n in enumerate(ns)]


def _zero_state(x, q) -> RodState:
    n = q.shape[0]
    return RodState(np.ascontiguousarray(x, dtype=np.float64), np.zeros((n + 1, 3)),
                    np.ascontiguousarray(q, dtype=np.float64), np.zeros((n, 3)))


# -------------------------------------------------------------------- configurations --

def load_dt_golden() -> dict:
    with open(DT_GOLDEN) as f:
        return json.load(f)


def _c0_material(n, L):
    l = L / n
    return dict(seg_len=np.full(n, l), radius=np.full(n, 0.01), young=np.full(n, 1e6),
                poisson=0.5, density=1000.0, damp_lin=0.1, damp_ang=0.1,
                gravity=(0.0, 0.0, -9.81))


def config0(dt: Optional[float] = None, n: int = 64) -> Workload:
    """Single extensible rod of 64 elements, clamped, sagging and swinging under gravity."""
    rng = np.random.default_rng(0)
    L = 1.0
    l = L / n
    x = np.zeros((n + 1, 3))
    x[:, 0] = np.arange(n + 1) * l
    x[1:, 1:] = rng.normal(0.0, 1e-3, size=(n, 2))
    q = frames_from_polyline(x)
    if dt is None:
        dt = load_dt_golden()["c0"]["dt"]
    spec = RodSpec(n=n, inextensible=False, n_iter=0, clamp=True, dt=float(dt),
                   clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]), **_c0_material(n, L))
    return Workload("c0: 1x64 extensible, static clamp, gravity", [(spec, _zero_state(x, q))],
                    n_steps=2000, steps_per_launch=100)


def config1(dt: Optional[float] = None, n: int = 512, static_clamp: bool = False,
            n_steps: int = 20000) -> Workload:
    """Two inextensible 512-element rods (catheter / guidewire-like), driven clamps."""
    rng = np.random.default_rng(1)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=4)
    if dt is None:
        dt = load_dt_golden()["c1"]["dt"]
    L = 1.0
    l = L / n
    freq = 2.0 / (20000 * dt)
    n_soft = int(math.ceil(0.05 * n))
    rods = []
    for k, (radius, young, base) in enumerate(((5e-4, 2e9, (0.0, 0.0, 0.0)),
                                               (2e-4, 5e10, (0.0, 5e-3, 0.0)))):
        E = np.full(n, young)
        if k == 1:
            E[n - n_soft:] = 5e9
        amp = 0.0 if static_clamp else l / 20.0
        tw = 0.0 if static_clamp else 0.2
        ph_x, ph_t = float(phases[2 * k]), float(phases[2 * k + 1])
        # clamp pose at t = 0 (input preparation: the prescribed trajectory sampled once)
        x_start = np.array(base) + np.array([amp * math.sin(ph_x), 0.0, 0.0])
        psi0 = tw * math.sin(ph_t)
        q_start = _qprod(_axis_angle((1.0, 0.0, 0.0), psi0), Q_ALONG_X)
        x = x_start[None, :] + np.outer(np.arange(n + 1) * l, [1.0, 0.0, 0.0])
        q = np.tile(q_start, (n, 1))
        spec = RodSpec(n=n, inextensible=True, n_iter=10, clamp=True, dt=float(dt),
                       gravity=(0.0, 0.0, -9.81), damp_lin=0.1, damp_ang=0.1, poisson=0.5,
                       density=1000.0, seg_len=np.full(n, l), radius=np.full(n, radius),
                       young=E, clamp_x0=tuple(base), clamp_q0=tuple(Q_ALONG_X),
                       clamp_amp=(amp, 0.0, 0.0), clamp_twist_amp=tw,
                       clamp_twist_axis=(1.0, 0.0, 0.0), clamp_freq=freq,
                       clamp_phase_x=ph_x, clamp_phase_twist=ph_t)
        rods.append((spec, _zero_state(x, q)))
    return Workload("c1: 2x512 inextensible, driven clamps, no contact", rods,
                    n_steps=n_steps, steps_per_launch=10)


def config5(one_way: bool, n: int = 512, shift: int = 128,
            n_steps: int = 20000) -> Tuple[Workload, np.ndarray]:
    """Catheter / guidewire pair bound together (Sec. 3.4 variants 1 and 2).

    The two rods of the 2 x 512 workload: rod 0 (catheter) keeps its driven clamp; rod 1
    (guidewire) is moved onto the catheter's axis with its static clamp `shift` elements behind
    the catheter's base, so its points shift + k coincide with the catheter's points k.  Returns
    the workload and the binding pairs (k, 4): (dependent rod, point, master rod, point) with the
    guidewire dependent, i.e. (1, k + shift, 0, k) for k = 1 .. n - shift.
    """
    wl = config1(n=n, n_steps=n_steps)
    (sa, sta), (sb, stb) = wl.rods
    l = float(sa.seg_len[0])
    base = sta.x[0] - np.array([shift * l, 0.0, 0.0])   # the catheter's base at t = 0
    x = base[None, :] + np.outer(np.arange(n + 1) * l, [1.0, 0.0, 0.0])
    q = np.tile(np.asarray(Q_ALONG_X, dtype=np.float64), (n, 1))
    sb = sb.replace(clamp_x0=tuple(base), clamp_q0=tuple(Q_ALONG_X), clamp_amp=(0.0, 0.0, 0.0),
                    clamp_twist_amp=0.0)
    k = np.arange(1, n - shift + 1)
    pairs = np.stack([np.ones_like(k), k + shift, np.zeros_like(k), k], axis=1).astype(np.int32)
    kind = "one-way" if one_way else "two-way"
    return (Workload("c5: catheter/guidewire 2x%d, %d %s bindings" % (n, len(k), kind),
                     [(sa, sta), (sb, _zero_state(x, q))], n_steps=n_steps, steps_per_launch=10),
            pairs)


def config6(n: int = 128, gap: float = 1e-3, dt: float = 0.0) -> Workload:
    """Two crossing rods for sphere contact: a stiff bar along x without gravity and a soft rod
    along y, `gap` above it where they cross (at their middles), that falls onto it.  Both 1 m,
    radius 1 cm, inextensible, static clamps.  dt = 0: set by the caller from the stability
    rule (the stricter of the two, shared by both)."""
    l = 1.0 / n
    r = 0.01
    rods = []
    q_y = (math.cos(math.pi / 4), -math.sin(math.pi / 4), 0.0, 0.0)   # third axis along +y
    for base, d3, q0, young, grav in (((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), Q_ALONG_X, 1e7,
                                       (0.0, 0.0, 0.0)),
                                      ((0.5, -0.5, 2 * r + gap), (0.0, 1.0, 0.0), q_y, 1e6,
                                       (0.0, 0.0, -9.81))):
        x = np.asarray(base)[None, :] + np.outer(np.arange(n + 1) * l, d3)
        q = np.tile(np.asarray(q0, dtype=np.float64), (n, 1))
        spec = RodSpec(n=n, inextensible=True, n_iter=10, clamp=True, dt=float(dt),
                       gravity=grav, damp_lin=0.5, damp_ang=0.5, poisson=0.5, density=1000.0,
                       seg_len=np.full(n, l), radius=np.full(n, r), young=np.full(n, young),
                       clamp_x0=tuple(base), clamp_q0=tuple(q0))
        rods.append((spec, _zero_state(x, q)))
    return Workload("c6: 2x%d crossing rods in sphere contact" % n, rods, n_steps=2000,
                    steps_per_launch=10)


def config2(n: int, inextensible: bool, dt: Optional[float] = None) -> Workload:
    """Single long rod with seeded initial curvature; element length 1/64 m."""
    rng = np.random.default_rng((2, n))
    l = 1.0 / 64.0
    x, q = curved_rod(n, l, rng, sigma=0.05)
    if dt is None:
        dt = load_dt_golden()["c0"]["dt"]
    spec = RodSpec(n=n, inextensible=inextensible, n_iter=10 if inextensible else 0,
                   clamp=True, dt=float(dt), clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]),
                   **_c0_material(n, n * l))
    kind = "inextensible" if inextensible else "extensible"
    return Workload("c2: 1x%d %s, curved, static clamp" % (n, kind), [(spec, _zero_state(x, q))],
                    n_steps=5000, steps_per_launch=10)


def config3(n_rods: int = 4096, n_min: int = 32, n_max: int = 2048) -> Workload:
    """Batch of uneven rods; each spec has dt = 0 (set from the stability rule by the caller)."""
    rng = np.random.default_rng(3)
    ns = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_rods))).astype(int)
    Es = np.exp(rng.uniform(math.log(1e6), math.log(1e10), size=n_rods))
    rs = rng.uniform(1e-4, 1e-3, size=n_rods)
    inext = np.zeros(n_rods, dtype=bool)
    inext[rng.permutation(n_rods)[: n_rods // 2]] = True
    l = 1.0 / 64.0
    rods = []
    geo = curved_rods(ns, l, rng, sigma=0.05)
    for r in range(n_rods):
        n = int(ns[r])
        x, q = geo[r]
        spec = RodSpec(n=n, inextensible=bool(inext[r]), n_iter=10 if inext[r] else 0,
                       clamp=True, dt=0.0, gravity=(0.0, 0.0, -9.81), damp_lin=0.1,
                       damp_ang=0.1, poisson=0.5, density=1000.0, seg_len=np.full(n, l),
                       radius=np.full(n, float(rs[r])), young=np.full(n, float(Es[r])),
                       clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
        rods.append((spec, _zero_state(x, q)))
    return Workload("c3: %d rods, N log-uniform [%d, %d], mixed variants" % (n_rods, n_min, n_max),
                    rods, n_steps=1000, steps_per_launch=1000)


def config4(n_rods: int = 256, n: int = 256, dt: float = 0.0) -> Workload:
    """Adjoint workload: curved and twisted inextensible rods of c0 material, L = 4 m.

    dt = 0 means "set from the stability rule by the caller" (as for c3)."""
    rng = np.random.default_rng(4)
    l = 4.0 / n
    rods = []
    for x, q in curved_rods([n] * n_rods, l, rng, sigma=0.05, twist_sigma=0.05):
        spec = RodSpec(n=n, inextensible=True, n_iter=10, clamp=True, dt=float(dt),
                       clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]), **_c0_material(n, n * l))
        rods.append((spec, _zero_state(x, q)))
    return Workload("c4: %dx%d inextensible adjoint rollout" % (n_rods, n), rods,
                    n_steps=400, steps_per_launch=20)


def tube_centreline(straight1: float = 0.3, bend_radius: float = 0.3,
                    bend_angle: float = 0.5 * math.pi, straight2: float = 0.5,
                    ds: float = 0.01) -> np.ndarray:
    """Centreline of a bent vessel in the horizontal plane: straight along x, an arc turning
    towards +y, straight again; points about ds apart."""
    pts = [np.array([s_, 0.0, 0.0]) for s_ in np.arange(0.0, straight1, ds)]
    c = np.array([straight1, bend_radius, 0.0])
    n_arc = max(2, int(math.ceil(bend_radius * bend_angle / ds)))
    for k in range(n_arc):
        a = bend_angle * k / n_arc
        pts.append(c + bend_radius * np.array([math.sin(a), -math.cos(a), 0.0]))
    end = c + bend_radius * np.array([math.sin(bend_angle), -math.cos(bend_angle), 0.0])
    tdir = np.array([math.cos(bend_angle), math.sin(bend_angle), 0.0])
    n_st = max(1, int(math.ceil(straight2 / ds)))
    for k in range(n_st + 1):
        pts.append(end + tdir * straight2 * k / n_st)
    return np.asarray(pts)


def tube_mesh(centre: np.ndarray, radius: float, n_around: int) -> np.ndarray:
    """Triangles (k, 3, 3) of a tube of the given radius around a centreline polyline: rings of
    n_around vertices (frames carried along by parallel transport), two triangles per quad,
    wound so that each face normal (b - a) x (c - a) points into the tube."""
    m = len(centre)
    t = np.gradient(centre, axis=0)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    u = np.zeros_like(centre)
    u0 = np.cross(t[0], [0.0, 0.0, 1.0])
    if np.linalg.norm(u0) < 1e-6:
        u0 = np.cross(t[0], [0.0, 1.0, 0.0])
    u[0] = u0 / np.linalg.norm(u0)
    for k in range(1, m):
        uk = u[k - 1] - np.dot(u[k - 1], t[k]) * t[k]
        u[k] = uk / np.linalg.norm(uk)
    w = np.cross(t, u)
    th = 2.0 * math.pi * np.arange(n_around) / n_around
    ring = centre[:, None, :] + radius * (np.cos(th)[None, :, None] * u[:, None, :]
                                          + np.sin(th)[None, :, None] * w[:, None, :])
    tris = []
    for k in range(m - 1):
        axis_mid = 0.5 * (centre[k] + centre[k + 1])
        for j in range(n_around):
            a, b = ring[k, j], ring[k, (j + 1) % n_around]
            c, d = ring[k + 1, (j + 1) % n_around], ring[k + 1, j]
            for tri in ((a, b, c), (a, c, d)):
                tri = np.array(tri)
                nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
                if np.dot(nrm, axis_mid - tri.mean(axis=0)) < 0:
                    tri = tri[[0, 2, 1]]
                tris.append(tri)
    return np.asarray(tris)


def _along(poly: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Points at arc lengths s along a polyline."""
    seg = np.linalg.norm(np.diff(poly, axis=0), axis=1)
    cum = np.r_[0.0, np.cumsum(seg)]
    out = np.empty((len(s), 3))
    for i, si in enumerate(s):
        k = min(np.searchsorted(cum, si, side="right") - 1, len(seg) - 1)
        f = (si - cum[k]) / seg[k]
        out[i] = poly[k] + f * (poly[k + 1] - poly[k])
    return out


def config7(n: int = 64, L: float = 1.0, rod_radius: float = 2e-3, young: float = 1e7,
            tube_radius: float = 1e-2, n_around: int = 12, dt: float = 0.0):
    """A straight-at-rest rod laid along the centreline of a bent vessel (procedural tube mesh)
    and clamped at its entrance: gravity and its own stiffness press it onto the wall.
    Returns (Workload, triangles (k, 3, 3))."""
    centre = tube_centreline()
    tris = tube_mesh(centre, tube_radius, n_around)
    x = _along(centre, np.linspace(0.0, L, n + 1))
    q = frames_from_polyline(x)
    seg = np.linalg.norm(np.diff(x, axis=0), axis=1)
    spec = RodSpec(n=n, inextensible=True, n_iter=10, clamp=True, dt=1.0, gravity=(0.0, 0.0, -9.81),
                   damp_lin=0.5, damp_ang=0.5, poisson=0.5, density=1000.0, seg_len=seg,
                   radius=np.full(n, rod_radius), young=np.full(n, young),
                   clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    if dt > 0:
        spec = spec.replace(dt=dt)
    return Workload("c7: %d-element rod in a bent tube (%d triangles)" % (n, len(tris)),
                    [(spec, _zero_state(x, q))], n_steps=400, steps_per_launch=10), tris


def straight_rod(n: int, L: float = 1.0, radius: float = 0.01, young: float = 1e6,
                 inextensible: bool = False, dt: float = 1e-5, gravity=(0.0, 0.0, -9.81),
                 damp: float = 0.0, n_iter: int = 10, clamp: bool = True,
                 q0=Q_ALONG_X) -> Tuple[RodSpec, RodState]:
    """Straight rod along the third axis of q0 with aligned frames (used by mechanics tests)."""
    l = L / n
    d3 = _third_axis(np.asarray(q0, dtype=np.float64))
    x = np.outer(np.arange(n + 1) * l, d3)
    q = np.tile(np.asarray(q0, dtype=np.float64), (n, 1))
    spec = RodSpec(n=n, inextensible=inextensible, n_iter=n_iter if inextensible else 0,
                   clamp=clamp, dt=dt, gravity=tuple(gravity), damp_lin=damp, damp_ang=damp,
                   poisson=0.5, density=1000.0, seg_len=np.full(n, l),
                   radius=np.full(n, radius), young=np.full(n, young),
                   clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    return spec, _zero_state(x, q)
