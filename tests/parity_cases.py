"""Inputs of the parity configurations that the GPU parity tests and the CPU test of the bars
share (seeded, synthetic; no GPU import)."""
import numpy as np

from paper_2509_04277_amd import workloads as W


def edge_rods(oracle):
    """Ragged rods (N = 1, 2, 3, 65, 130, 200), both variants, clamped (driven) and free,
    external loads, intrinsic shape, non-uniform material, random initial velocities."""
    rng = np.random.default_rng(40)
    rods = []
    for n, inext, clamp in ((1, False, True), (2, True, True), (3, False, False), (65, True, True),
                            (130, False, True), (200, True, False)):
        x, q = W.curved_rod(n, 0.02, rng, sigma=0.2, twist_sigma=0.1)
        spec = W.RodSpec(
            n=n, inextensible=inext, n_iter=7 if inext else 0, clamp=clamp, dt=2e-5,
            gravity=(0.5, -2.0, -9.81), damp_lin=0.3, damp_ang=0.2, poisson=0.35, density=1100.0,
            seg_len=rng.uniform(0.015, 0.025, n), radius=rng.uniform(0.004, 0.006, n),
            young=rng.uniform(2e5, 1e6, n), kp_scale=0.8, bend_scale=1.2, twist_scale=0.9,
            u_hat=rng.normal(0, 1.0, (n - 1, 3)) if n > 1 else None,
            f_ext=rng.normal(0, 1e-3, (n + 1, 3)), tau_ext=rng.normal(0, 1e-5, (n, 3)),
            clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]),
            clamp_amp=(0.0, 1e-3, 5e-4) if clamp else (0, 0, 0), clamp_twist_amp=0.1 if clamp else 0,
            clamp_twist_axis=(0.2, 0.0, 1.0), clamp_freq=7.0, clamp_phase_x=0.3,
            clamp_phase_twist=1.3)
        st = W.RodState(x, rng.normal(0, 1e-2, (n + 1, 3)), q, rng.normal(0, 0.1, (n, 3)))
        if clamp:
            xc, qc, _ = oracle.Rod(spec).clamp_pose(0.0)
            st.x = st.x - st.x[0] + xc
            st.q[0] = qc
        rods.append((spec, st))
    return rods


# ---------------------------------------------------------------- bound and touching rods --

class GroupCase:
    """Rods stepped together through bindings or contact (Sec. 3.4, Sec. 2.3): the handle's
    rods, how the handle is set up, and the same problem for the oracle's group step, whose
    rods come in `order` (for bindings the dependent rod first, the master second)."""

    def __init__(self, rods, n_steps, window, bars, bind=None, contact=None):
        self.rods = [(fp32_radius(s), st) for s, st in rods]
        self.n_steps, self.window, self.bars = n_steps, window, bars
        self.bind, self.contact = bind, contact
        if bind is not None:
            pairs, one_way = bind
            self.order = [int(pairs[0, 0]), int(pairs[0, 2])]
            self.oracle_kw = dict(pairs=np.stack([pairs[:, 1], pairs[:, 3]], 1), one_way=one_way)
        else:
            self.order = list(range(len(rods)))
            self.oracle_kw = dict(mu=contact[1])

    def setup(self, batch):
        """Bindings or contact on a RodBatch of self.rods."""
        if self.bind is not None:
            batch.set_bindings(*self.bind)
        else:
            batch.set_contact(*self.contact)


def fp32_radius(spec):
    """The spec with its element radii rounded to FP32 (kept as doubles), as the GPU receives
    them: contact decides on distances against sums of radii, and where touching rods rest a
    radius rounding (a few 1e-10 m) is not small against a step's sinking."""
    return spec.replace(radius=np.asarray(spec.radius, dtype=np.float32).astype(np.float64))


def _dt_shared(oracle, rods):
    """The stricter of the rods' stable time steps (the oracle's rule), given to all of them."""
    dt = min(oracle.Rod(s.replace(dt=1.0)).dt_rule() for s, _ in rods)
    return [(s.replace(dt=dt), st) for s, st in rods]


def bound_pair(one_way):
    """The catheter / guidewire pair (both 512 elements, 384 bound points)."""
    wl, pairs = W.config5(one_way)
    return GroupCase(wl.rods, 500, 10, "c5", bind=(pairs, one_way))


def crossing(oracle, mu):
    """Two crossing 128-element rods: a stiff bar and a soft rod falling across its middle."""
    return GroupCase(_dt_shared(oracle, W.config6().rods), 2000, 10, None, contact=([[0, 1]], mu))


def coiled(oracle, n=48, turns=2, L=1.0, r=0.01, rise=0.5):
    """Two flat turns of a circle with a slight helical rise (the second turn rise x 2r above
    the first); the rest shape is this shape.  Self-contact, friction 0.2."""
    R_ = L / (2 * np.pi * turns)
    s = np.linspace(0.0, L, n + 1)
    x = np.stack([R_ * np.sin(s / R_), R_ * (1 - np.cos(s / R_)), rise * 2 * r * s / (L / turns)], 1)
    q = W.frames_from_polyline(x)
    spec, st = W.straight_rod(n, L=L, radius=r, inextensible=True, dt=1e-5, gravity=(0, 0, 0),
                              damp=5.0)
    rod = oracle.Rod(spec)
    u_hat = np.array([rod.darboux(q, j) for j in range(n - 1)])
    lens = np.linalg.norm(x[1:] - x[:-1], axis=1)
    spec = spec.replace(u_hat=u_hat, seg_len=lens, clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    st = st.copy()
    st.x, st.q = x, q
    return GroupCase(_dt_shared(oracle, [(spec, st)]), 200, 10, None, contact=([[0, -1]], 0.2))


def side_by_side(oracle, n=64, r=0.01):
    """Two parallel rods whose elements are much shorter than their radius (l = 0.08 r), one
    pressed sideways onto the other by gravity; friction 0.2."""
    L = n * 0.08 * r
    a, sa = W.straight_rod(n, L=L, radius=r, young=1e7, inextensible=True, gravity=(0, 0, 0),
                           damp=0.5)
    b, sb = W.straight_rod(n, L=L, radius=r, young=1e6, inextensible=True,
                           gravity=(0, -9.81, 0), damp=0.5)
    off = np.array([0.0, 1.99 * r, 0.0])
    sb = sb.copy()
    sb.x = sb.x + off
    b = b.replace(clamp_x0=tuple(np.asarray(b.clamp_x0) + off))
    return GroupCase(_dt_shared(oracle, [(a, sa), (b, sb)]), 400, 10, None,
                     contact=([[0, 1]], 0.2))


def unequal(oracle, gap=1e-3):
    """A 300-element bar along x (1 m, no gravity) and a 60-element rod along y (0.5 m) that
    falls across its middle from gap above; both radius 4 mm, inextensible, static clamps,
    friction 0.2."""
    import math
    r = 0.004
    out = []
    q_y = (math.cos(math.pi / 4), -math.sin(math.pi / 4), 0.0, 0.0)
    for n, L, base, d3, q0, young, grav in (
            (300, 1.0, (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), W.Q_ALONG_X, 1e7, (0.0, 0.0, 0.0)),
            (60, 0.5, (0.5, -0.25, 2 * r + gap), (0.0, 1.0, 0.0), q_y, 1e6, (0.0, 0.0, -9.81))):
        l = L / n
        x = np.asarray(base)[None, :] + np.outer(np.arange(n + 1) * l, d3)
        q = np.tile(np.asarray(q0, dtype=np.float64), (n, 1))
        spec = W.RodSpec(n=n, inextensible=True, n_iter=10, clamp=True, dt=1e-5, gravity=grav,
                         damp_lin=0.5, damp_ang=0.5, poisson=0.5, density=1000.0,
                         seg_len=np.full(n, l), radius=np.full(n, r), young=np.full(n, young),
                         clamp_x0=tuple(base), clamp_q0=tuple(q0))
        out.append((spec, W.RodState(x=x, v=np.zeros_like(x), q=q, w=np.zeros((n, 3)))))
    return GroupCase(_dt_shared(oracle, out), 1500, 10, None, contact=([[0, 1]], 0.2))


def group_cases(oracle):
    """The bound and touching configurations of the parity tests, by name."""
    return {"c5-one": bound_pair(True), "c5-two": bound_pair(False),
            "c6-mu0": crossing(oracle, 0.0), "c6-mu0.3": crossing(oracle, 0.3),
            "coiled": coiled(oracle), "side": side_by_side(oracle), "unequal": unequal(oracle)}


def group_run(oracle, case, n_steps, states=None, t0=0.0, round_mask=0, specs=None, **kw):
    """The oracle's group step over n_steps from `states` (default: the FP32 input), in the
    handle's rod order; returns (states, largest number of contacts of one point).  specs and
    kw replace the case's rods' specs and group arguments."""
    specs = [s for s, _ in case.rods] if specs is None else specs
    if states is None:
        states = [_fp32(st) for _, st in case.rods]
    okw = dict(case.oracle_kw, **kw)
    o = case.order
    out, most = oracle.rollout_group([specs[i] for i in o], [states[i] for i in o], n_steps,
                                     t0=t0, round_mask=round_mask, **okw)
    res = [None] * len(o)
    for j, i in enumerate(o):
        res[i] = out[j]
    return res, most


def group_window(oracle, case, n_steps, k, round_mask=0, specs=None, **kw):
    """Oracle states after n_steps - k and n_steps steps (handle order), and the most
    contacts of one point over the run."""
    specs = [s for s, _ in case.rods] if specs is None else specs
    a, most_a = group_run(oracle, case, n_steps - k, round_mask=round_mask, specs=specs, **kw)
    b, most_b = group_run(oracle, case, k, states=a, t0=(n_steps - k) * specs[0].dt,
                          round_mask=round_mask, specs=specs, **kw)
    return a, b, max(most_a, most_b)


def _fp32(st):
    out = st.copy()
    for f in ("x", "v", "q", "w"):
        setattr(out, f, np.asarray(getattr(st, f), dtype=np.float32).astype(np.float64))
    return out


# ------------------------------------------------------------------ environment collision --

class EnvCase:
    """One rod against a static triangle mesh (Sec. 2.2) with friction mu; the mesh as both
    sides receive it (vertices rounded to FP32)."""

    def __init__(self, spec, state, tris, mu, n_steps, window, bars):
        self.rods = [(fp32_radius(spec), state)]
        self.tris = np.asarray(tris, dtype=np.float32).astype(np.float64)
        self.mu, self.n_steps, self.window, self.bars = mu, n_steps, window, bars


def tube(oracle, mu):
    """The environment workload: a 64-element rod laid along a bent tube's axis, clamped at
    its entrance, pressed onto the wall by gravity and its own stiffness."""
    wl, tris = W.config7(n=64)
    (spec, st), = _dt_shared(oracle, wl.rods)
    return EnvCase(spec, st, tris, mu, 1200, 10, "tube")


def floor_plane(z=0.0, size=2.0):
    a, b, c, d = ([-size, -size, z], [size, -size, z], [size, size, z], [-size, size, z])
    return np.array([[a, b, c], [a, c, d]], dtype=np.float64)


def on_floor(oracle, inext):
    """A clamped 32-element rod that sags onto a floor just below it and slides on it with
    friction 0.4."""
    spec, st = W.straight_rod(32, L=0.5, radius=0.01, inextensible=inext, dt=1e-5, damp=0.5)
    (spec, st), = _dt_shared(oracle, [(spec, st)])
    return EnvCase(spec, st, floor_plane(z=-0.02), 0.4, 1500, 10, "floor")


def env_run(oracle, case, n_steps, state=None, t0=0.0, round_mask=0):
    """The oracle's rod against the case's mesh over n_steps from `state` (default: the FP32
    input); with round_mask, the fields of the mask rounded to FP32 after every step."""
    spec = case.rods[0][0]
    env = oracle.Env(case.tris, case.mu)
    st = _fp32(case.rods[0][1]) if state is None else state
    if not round_mask:
        return oracle.rollout_env(spec, st, n_steps, env, t0=t0)
    most = 0
    for k in range(n_steps):
        st, m = oracle.rollout_env(spec, st, 1, env, t0=t0 + k * spec.dt)
        st = _round(st, round_mask)
        most = max(most, m)
    return st, most


def env_window(oracle, case, n_steps, k, round_mask=0):
    """Oracle states after n_steps - k and n_steps steps, and the most colliding points."""
    spec = case.rods[0][0]
    a, m1 = env_run(oracle, case, n_steps - k, round_mask=round_mask)
    b, m2 = env_run(oracle, case, k, state=a, t0=(n_steps - k) * spec.dt, round_mask=round_mask)
    return [a], [b], max(m1, m2)


def _round(st, mask):
    out = st.copy()
    for f, bit in (("x", 1), ("v", 2), ("q", 4), ("w", 8)):
        if mask & bit:
            setattr(out, f, np.asarray(getattr(st, f), dtype=np.float32).astype(np.float64))
    return out


def env_restarts(oracle, case, states, stops, k=10):
    """From each state states[i] (taken at step stops[i] of a run), k steps of the oracle: the
    plain run, and runs that show how far FP32-sized differences of the state carry over the
    window (its floor): v, q and w rounded to FP32 after every step; a start whose v, q and w
    are moved by 2^-22 relative; a start whose positions are moved by 2^-24 relative (half an
    FP32 ulp).  Signs are seeded by the step.  Contacts (touching or not, sticking or slipping)
    make some windows far more sensitive than others, and stiff rods answer a position change
    far more than a velocity change; the moved starts show that where the rounding alone does
    not.  Returns [(start, plain, [perturbed runs])]."""
    spec = case.rods[0][0]
    out = []
    for st, s in zip(states, stops):
        st = _round(st, 15)
        b, _ = env_run(oracle, case, k, state=st, t0=s * spec.dt)
        pert = [env_run(oracle, case, k, state=st, t0=s * spec.dt, round_mask=14)[0]]
        for m in _moved_starts(st, s):
            pert.append(env_run(oracle, case, k, state=m, t0=s * spec.dt)[0])
        out.append((st, b, pert))
    return out


def _moved(st, seed, fields=("v", "q", "w"), scale=2.0 ** -22):
    rng = np.random.default_rng(seed)
    out = st.copy()
    for f in fields:
        a = np.asarray(getattr(st, f), dtype=np.float64)
        setattr(out, f, a * (1.0 + rng.choice([-1.0, 1.0], a.shape) * scale))
    return out


def _moved_starts(st, seed):
    return [_moved(st, seed), _moved(st, seed + 1, ("x",), 2.0 ** -24)]


def rod_restarts(oracle, spec, states, stops, k=10):
    """As env_restarts, for a rod on its own."""
    r = oracle.Rod(spec)
    out = []
    for st, s in zip(states, stops):
        st = _round(st, 15)
        b = r.rollout(st, k, t0=s * spec.dt)[0]
        pert = [r.rollout_rounded(st, k, 14, t0=s * spec.dt)]
        pert += [r.rollout(m, k, t0=s * spec.dt)[0] for m in _moved_starts(st, s)]
        out.append((st, b, pert))
    return out


def window_floor(spec, x0, start, plain, perturbed, k, errors):
    """Floor of one restart window: per quantity the largest difference of a perturbed run
    from the plain run (errors: parity_metrics.errors)."""
    t = lambda u: (u.x, u.v, u.q, u.w)
    fl = [errors(spec, x0, t(start), t(p), t(start), t(plain), k) for p in perturbed]
    out = {m: max(f[m] for f in fl) for m in fl[0]}
    out.pop("unit")
    return out


def env_changed(case, spec=None, mu=None):
    """The case with another spec or friction coefficient (same input and mesh)."""
    c = EnvCase(case.rods[0][0] if spec is None else spec, case.rods[0][1], case.tris,
                case.mu if mu is None else mu, case.n_steps, case.window, case.bars)
    c.tris = case.tris
    return c


# ------------------------------------------------------- internal friction, haptic pose --

def damped(oracle, n, inext, td_over_dt, seed=6):
    """A curved, twisted clamped rod released under gravity with internal friction tau_d a
    multiple of the stable dt (the dashpots then take part in the stability rule)."""
    rng = np.random.default_rng(seed)
    x, q = W.curved_rod(n, 1.0 / n, rng, 0.05, twist_sigma=0.05)
    spec, _ = W.straight_rod(n, inextensible=inext, dt=1e-5)
    spec = spec.replace(seg_len=np.linalg.norm(np.diff(x, axis=0), axis=1), clamp_x0=tuple(x[0]),
                        clamp_q0=tuple(q[0]))
    dt0 = oracle.Rod(spec.replace(dt=1.0)).dt_rule()
    spec = spec.replace(damp_int=td_over_dt * dt0)
    spec = spec.replace(dt=oracle.Rod(spec.replace(dt=1.0)).dt_rule())
    return spec, W.RodState(x=x, v=np.zeros_like(x), q=q, w=np.zeros((n, 3)))


def swinging(oracle, n, inext, seed=3):
    """A clamped horizontal rod released under gravity, slightly perturbed."""
    spec, st = W.straight_rod(n, inextensible=inext, dt=1e-5, damp=0.3)
    spec = spec.replace(dt=oracle.Rod(spec.replace(dt=1.0)).dt_rule())
    rng = np.random.default_rng(seed)
    st = st.copy()
    st.x = st.x + rng.normal(0, 1e-4, st.x.shape) * np.r_[0.0, np.ones(n)][:, None]
    return spec, st


# ----------------------------------------------------------------------- uneven batches --

def with_rule_dt(oracle, rods):
    """Each rod at its own stable time step (the oracle's rule)."""
    return [(s.replace(dt=oracle.Rod(s.replace(dt=1.0)).dt_rule()), st) for s, st in rods]


def batch48(oracle):
    """48 uneven rods (N 8..700, both variants), per-rod dt: several kernel-shape buckets."""
    return with_rule_dt(oracle, W.config3(n_rods=48, n_min=8, n_max=700).rods)


def c3_pick(rods):
    """Sampled rods of the 4096-rod batch: every 256th, the costliest (longest inextensible)
    and the shortest."""
    ns = np.array([s.n for s, _ in rods])
    cost = ns * np.array([4 + s.n_iter for s, _ in rods])
    return sorted(set(range(0, len(rods), 256)) | {int(np.argmax(cost)), int(np.argmin(ns))})


def group_restarts(oracle, case, states, stops, k=10):
    """As env_restarts, for rods stepped together: states[i] holds the rods' states (handle
    order) at step stops[i]; returns [(starts, plain, rounded, moved)], each a list over the
    rods."""
    dt = case.rods[0][0].dt
    out = []
    for sts, s in zip(states, stops):
        sts = [_round(st, 15) for st in sts]
        b, _ = group_run(oracle, case, k, states=sts, t0=s * dt)
        pert = [group_run(oracle, case, k, states=sts, t0=s * dt, round_mask=14)[0]]
        moved = [_moved_starts(st, 97 * s + 2 * i) for i, st in enumerate(sts)]
        for j in range(len(moved[0])):
            pert.append(group_run(oracle, case, k, states=[m[j] for m in moved], t0=s * dt)[0])
        out.append((sts, b, pert))
    return out


def group_floor(case, x0s, start, plain, perturbed, k, errors):
    """Floor of one restart window of a group: per quantity the largest over the rods of
    window_floor (perturbed: the perturbed runs, each a list over the rods)."""
    fl = [window_floor(spec, x0, a, b, [p[r] for p in perturbed], k, errors)
          for r, ((spec, _), x0, a, b) in enumerate(zip(case.rods, x0s, start, plain))]
    return {m: max(f[m] for f in fl) for m in fl[0]}


# restart steps of the touching configurations (their runs' lengths: the stops' last + 10)
TOUCHING_STOPS = {"c6-mu0": (500, 1000, 1500, 1990), "c6-mu0.3": (500, 1000, 1500, 1990),
                  "coiled": (100, 190), "side": (200, 390), "unequal": (500, 1000, 1490)}
