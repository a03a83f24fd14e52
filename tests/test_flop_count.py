"""The method's floating-point operation count per element-step (the figure the benchmark
prices its ALU roofline with), pinned by evaluating one step with numbers that count their own
arithmetic: the counted step must reproduce the oracle's step (to rounding), so the counted
operations are the ones the method needs, and each part's count must equal the benchmark's
table.  Conventions: +, -, x one operation each (a multiply-add two), reciprocal square root
one, a sign change none; per-element material coefficients (computed once per rod) and plain
constants are not counted.

The parts (Sec. 2.1): segment forces and penalty torque (eqs. (2), (7)-(8)), joint moments
from the relative rotation of neighbouring frames (eqs. (3), (5)-(6)), their accumulation on
points and frames, force and torque integration (Euler's equations with damping), one
distance-constraint impulse per segment and iteration (red-black sweeps), and the velocity
integration with the quaternion renormalised."""
import math

import numpy as np
import pytest

import bench
from oracle import oracle as O
from paper_2509_04277_amd import workloads as W

_OPS = [0]


def _val(o):
    return o.v if isinstance(o, Num) else o


class Num:
    """A float that counts the arithmetic done on it."""
    __slots__ = ("v",)

    def __init__(self, v):
        self.v = float(v)

    def _op(self, r):
        _OPS[0] += 1
        return Num(r)

    def __add__(a, b): return a._op(a.v + _val(b))
    def __radd__(a, b): return a._op(_val(b) + a.v)
    def __sub__(a, b): return a._op(a.v - _val(b))
    def __rsub__(a, b): return a._op(_val(b) - a.v)
    def __mul__(a, b): return a._op(a.v * _val(b))
    def __rmul__(a, b): return a._op(_val(b) * a.v)
    def __neg__(a): return Num(-a.v)


def rsqrt(a):
    _OPS[0] += 1
    return Num(1.0 / math.sqrt(a.v))


def add(a, b): return tuple(x + y for x, y in zip(a, b))
def sub(a, b): return tuple(x - y for x, y in zip(a, b))
def scale(s, a): return tuple(s * x for x in a)


def dot(a, b):
    r = a[0] * b[0]
    for x, y in zip(a[1:], b[1:]):
        r = r + x * y
    return r


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def segment(xa, xb, q, c):
    """Segment vector e, force f on the segment's far point, penalty torque (body x, y) on its
    frame: f = (l K_p / |e|) (d3 - (t . d3) t) [- (K_s / l)(|e| - l) t], torque l K_p e3 x R^T t."""
    e = sub(xb, xa)
    len2 = dot(e, e)
    il = rsqrt(len2)
    t = scale(il, e)
    w, x, y, z = q
    ww, xx, yy, zz = w * w, x * x, y * y, z * z
    xy, xz, yz, wx, wy, wz = x * y, x * z, y * z, w * x, w * y, w * z
    d1 = (ww + xx - yy - zz, 2.0 * (xy + wz), 2.0 * (xz - wy))
    d2 = (2.0 * (xy - wz), ww - xx + yy - zz, 2.0 * (yz + wx))
    d3 = (2.0 * (xz + wy), 2.0 * (yz - wx), ww - xx - yy + zz)
    f = scale(c["lkp"] * il, sub(d3, scale(dot(t, d3), t)))
    if not c["inext"]:
        f = sub(f, scale(c["ks_l"] * (len2 * il - c["l"]), t))
    return e, f, (-(c["lkp"] * dot(d2, t)), c["lkp"] * dot(d1, t))


def joint(qa, qb, c):
    """Body torques on frames j and j+1 from m = K (u - u_hat), u = (2 / lbar) vec(conj(q_j) q_{j+1})."""
    rw = dot(qa, qb)
    va, vb = qa[1:], qb[1:]
    rv = sub(sub(scale(qa[0], vb), scale(qb[0], va)), cross(va, vb))
    m = (c["C1"] * rv[0] - c["D"][0], c["C1"] * rv[1] - c["D"][1], c["C3"] * rv[2] - c["D"][2])
    rwm, rxm = scale(rw, m), cross(rv, m)
    return add(rwm, rxm), sub(rxm, rwm)


def point_update(v, F, c, g):
    return add(v, scale(c["dt"], add(scale(c["winv"], F), sub(g, scale(c["dl"], v)))))


def frame_update(o, tau, c):
    al = (c["i1"] * tau[0] - c["kg"] * (o[1] * o[2]) - c["da"] * o[0],
          c["i1"] * tau[1] + c["kg"] * (o[0] * o[2]) - c["da"] * o[1],
          c["i3"] * tau[2] - c["da"] * o[2])
    return add(o, scale(c["dt"], al))


def impulse(e, va, vb, wa, wb, cs):
    """lambda n = ci (1 - l / |d|) d at the predicted d = e + dt (v_b - v_a)."""
    d = add(e, scale(cs["dt"], sub(vb, va)))
    im = scale(cs["ci"] - cs["cil"] * rsqrt(dot(d, d)), d)
    return add(va, scale(wa, im)), sub(vb, scale(wb, im))


def advance(x, v, q, o, dt):
    dq = (-dot(q[1:], o),) + add(scale(q[0], o), cross(q[1:], o))
    q2 = add(q, scale(0.5 * dt, dq))
    return add(x, scale(dt, v)), scale(rsqrt(dot(q2, q2)), q2)


def coefficients(spec):
    """Per-element constants of the material model (computed once per rod, not counted)."""
    n, nu = spec.n, spec.poisson
    el = []
    for j in range(n):
        l, r, E = float(spec.seg_len[j]), float(spec.radius[j]), float(spec.young[j])
        G = E / (2 * (1 + nu))
        A = math.pi * r * r
        m = spec.density * A * l
        I1, I3 = m * (3 * r * r + l * l) / 12, m * r * r / 2
        el.append(dict(l=l, m=m, lkp=l * spec.kp_scale * G * A, ks_l=E * A / l,
                       inext=spec.inextensible, K1=spec.bend_scale * E * math.pi * r ** 4 / 4,
                       K3=spec.twist_scale * G * math.pi * r ** 4 / 2,
                       i1=1 / I1, i3=1 / I3, kg=(I3 - I1) / I1, da=spec.damp_ang, dt=spec.dt))
    jt = []
    for j in range(n - 1):
        lbar = 0.5 * (el[j]["l"] + el[j + 1]["l"])
        K1 = 0.5 * (el[j]["K1"] + el[j + 1]["K1"])
        K3 = 0.5 * (el[j]["K3"] + el[j + 1]["K3"])
        uh = spec.u_hat[j] if spec.u_hat is not None else (0.0, 0.0, 0.0)
        jt.append(dict(C1=2 * K1 / lbar, C3=2 * K3 / lbar, D=(K1 * uh[0], K1 * uh[1], K3 * uh[2])))
    winv = []
    for i in range(n + 1):
        M = (0.5 * el[i - 1]["m"] if i > 0 else 0.0) + (0.5 * el[i]["m"] if i < n else 0.0)
        winv.append(0.0 if (spec.clamp and i == 0) else 1 / M)
    cs = []
    for j in range(n):
        ci = 1 / (spec.dt * (winv[j] + winv[j + 1]))
        cs.append(dict(ci=ci, cil=ci * el[j]["l"], dt=spec.dt))
    return el, jt, winv, cs


def counted_step(spec, st, probe):
    """One step of a rod with a static clamp; returns the new state and, per part, the
    operations spent on element `probe` (its segment, joint, point probe + 1 and frame)."""
    n = spec.n
    el, jt, winv, cs = coefficients(spec)
    counts = {}

    def run(part, j, fn, *a):
        c0 = _OPS[0]
        r = fn(*a)
        if j == probe:
            counts[part] = counts.get(part, 0) + _OPS[0] - c0
        return r

    nums = lambda rows: [tuple(Num(c) for c in r) for r in rows]
    x, v, q, w = nums(st.x), nums(st.v), nums(st.q), nums(st.w)
    g = tuple(float(c) for c in spec.gravity)
    E, F, TP, TJ, TN = [], [], [], [], []
    for j in range(n):
        e, f, tp = run("segment", j, segment, x[j], x[j + 1], q[j], el[j])
        E.append(e); F.append(f); TP.append(tp)
    for j in range(n - 1):
        tj, tn = run("joint", j, joint, q[j], q[j + 1], jt[j])
        TJ.append(tj); TN.append(tn)

    def force_on(i):   # point i >= 1: pulled by segment i - 1, pushed back by segment i
        return sub(F[i - 1], F[i]) if i < n else F[i - 1]

    def torque_on(j):
        own = ((TP[j][0] + TJ[j][0], TP[j][1] + TJ[j][1], TJ[j][2]) if j < n - 1
               else (TP[j][0], TP[j][1], Num(0.0)))
        return add(own, TN[j - 1]) if j > 0 else own

    Fp = {i: run("accumulate", i - 1, force_on, i) for i in range(1, n + 1)}
    Tf = {j: run("accumulate", j, torque_on, j) for j in range(n)}
    for i in range(1, n + 1):
        v[i] = run("point", i - 1, point_update, v[i], Fp[i],
                   dict(winv=winv[i], dl=spec.damp_lin, dt=spec.dt), g)
    for j in range(1, n):
        w[j] = run("frame", j, frame_update, w[j], Tf[j], el[j])
    for it in range(spec.n_iter if spec.inextensible else 0):
        for parity in (0, 1):
            for j in range(parity, n, 2):
                v[j], v[j + 1] = run("impulse", j, impulse, E[j], v[j], v[j + 1], winv[j],
                                     winv[j + 1], cs[j])
    for j in range(n):
        x[j + 1], q[j] = run("advance", j, advance, x[j + 1], v[j + 1], q[j], w[j], spec.dt)
    q[0] = tuple(Num(c) for c in spec.clamp_q0)
    arr = lambda rows: np.array([[c.v for c in r] for r in rows])
    return (arr(x), arr(v), arr(q), arr(w)), counts


def _rod(inext, n=9, seed=3):
    """A bent, twisted, moving rod: every term of the step is active."""
    spec, st = W.straight_rod(n, inextensible=inext, dt=2e-5, damp=0.3)
    rng = np.random.default_rng(seed)
    st.x[1:] += rng.normal(0, 0.02, st.x[1:].shape)
    st.v[1:] = rng.normal(0, 0.1, st.v[1:].shape)
    q = st.q + rng.normal(0, 0.05, st.q.shape)
    q[0] = st.q[0]
    st.q = q / np.linalg.norm(q, axis=1, keepdims=True)
    st.w[1:] = rng.normal(0, 1.0, st.w[1:].shape)
    return spec, st


@pytest.mark.parametrize("inext", [True, False])
def test_counted_step_is_the_oracle_step(inext):
    spec, st = _rod(inext)
    got, _ = counted_step(spec, st, probe=3)
    ref, _ = O.Rod(spec).rollout(st, 1)
    for a, b, name in zip(got, (ref.x, ref.v, ref.q, ref.w), "xvqw"):
        err = np.abs(a - b).max() / np.abs(b).max()
        assert err < 1e-12, (name, err)
    # the step moved every field, so the comparison sees each part
    for a, b in zip(got, (st.x, st.v, st.q, st.w)):
        assert np.abs(a - b).max() > 1e-9


@pytest.mark.parametrize("inext", [True, False])
@pytest.mark.parametrize("probe", [2, 5])
def test_part_counts_are_the_benchmark_table(inext, probe):
    spec, st = _rod(inext)
    _, counts = counted_step(spec, st, probe)
    table = bench.FLOPS_PER_ROW
    seg = table["segment"] + (0 if inext else table["stretch"])
    assert counts["segment"] == seg
    for part in ("joint", "accumulate", "point", "frame", "advance"):
        assert counts[part] == table[part], part
    if inext:
        assert counts["impulse"] == table["impulse"] * spec.n_iter
    else:
        assert "impulse" not in counts
    assert sum(counts.values()) == bench.flops_per_element_step(inext, spec.n_iter)


def test_headline_and_batch_counts():
    """535 operations per element-step for an inextensible rod at 10 constraint iterations,
    224 for an extensible one."""
    assert bench.flops_per_element_step(True, 10) == 535
    assert bench.flops_per_element_step(False, 0) == 224
