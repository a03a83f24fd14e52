"""Whole-state parity metrics shared by the GPU parity tests and the CPU test that shows each
bar can fail (a 10 % change of one coefficient of the method, made in the oracle, must break
at least one bar on the configurations that cover it).

Compared quantities, GPU (FP32) against the oracle (FP64), after a run and over a window of
its last k steps:
  x     positions, max over points of |dx|, relative to the largest displacement of a point
        over the run (small when nothing moves much: floored at 1e-3 of the rod length);
  tip   |dx| of the last point, against 1e-4 of the rod length (the method's target);
  q     frames, max |dq| over frames after aligning the sign of each quaternion;
  u     Darboux vectors u_j = (2 / lbar_j) vec(conj(q_j) q_{j+1}) (eqs. (5)-(6)), max |du|
        relative to max |u| of the oracle (floored at 1 / rod length);
  vbar  window-mean point velocities (x(T) - x(T-k)) / (k dt), relative to their max (floored
        at 1e-3 of the rod length per window), robust to stiff-mode noise in v itself;
  wbar  window-mean body rates 2 vec(conj(q(T-k)) q(T)) / (k dt), relative likewise (floored
        at 1e-3 rad per window);
  unit  max | |q| - 1 | of the GPU frames.
No GPU import here: the module runs on the CPU too.
"""
import numpy as np

# Base bars per quantity (see the module docstring for the normalisations); the tip's is the
# method's target, 1e-4 of the rod length.
TOL = {"x": 1e-3, "tip": 1e-4, "q": 1e-4, "u": 1e-3, "vbar": 1e-3, "wbar": 1e-3, "unit": 1e-6}

# FP32 floor of a configuration: the same metrics between the oracle and the oracle with v, q
# and w rounded to FP32 after every step (x kept exact: the GPU holds positions as pairs of
# floats, and its frames carry FP32-size errors from the quaternion and torque arithmetic of
# every step, which the rounding of q stands for).  Bar of a quantity on a configuration =
# max(base bar, 10 x floor) rounded up to two digits: the factor covers the several roundings
# of a step's arithmetic.  test_parity_bars recomputes the floors and checks these numbers.
# A stiff configuration run at half its stability limit keeps the noise that enters its stiff
# modes (symplectic Euler does not damp them): the two-instrument pair's floors grow with the
# run's length, hence its 2000-step and 20000-step bars.  The bound pair is compared at 500
# steps, before its free guidewire section (straight, compressed by the catheter's drive)
# buckles in a direction that rounding decides.  Runs in which contacts switch (touching rods,
# rods against a mesh) are held in short windows restarted from the GPU's state instead, to
# bars from each window's own floor (floor_bars).
FLOOR_FACTOR = 10.0
BARS = {
    "c0": TOL,
    "c0-swing": TOL,
    "c1": dict(TOL, u=1.3e-2, wbar=2.9e-2),                                  # 2000 steps
    "c1-full": dict(TOL, x=1.6e-2, q=1.8e-3, u=5.4e-1, wbar=1.1e-1),          # 20000 steps
    "edge": dict(TOL, q=1.2e-4),
    "c2": dict(TOL, wbar=1.9e-3),                                              # 4096, 5000 steps
    "damped": dict(TOL, wbar=1.5e-3),                                          # 600 steps
    "batch": dict(TOL, wbar=8.1e-3),                                           # 48 rods, 150
    "c3": dict(TOL, wbar=9.6e-3),                                              # sampled, 1000
    "c5": dict(TOL, u=1.2e-2, wbar=1.5e-2),                                   # bound pair, 500
}


def fp32_input(st):
    """The state as the GPU receives it: every value rounded to FP32 (kept as doubles), so that
    the oracle starts from exactly the GPU's input.  (On a metres-long rod the FP32 rounding of
    the initial positions alone moves frames by up to 1e-3 after a few hundred steps.)"""
    out = st.copy()
    for k in ("x", "v", "q", "w"):
        setattr(out, k, np.asarray(getattr(st, k), dtype=np.float32).astype(np.float64))
    return out


def fp32_rods(rods):
    """fp32_input of every (spec, state) pair."""
    return [(s, fp32_input(st)) for s, st in rods]


def _qalign(q, ref):
    s = np.sign(np.sum(q * ref, axis=1))
    s[s == 0] = 1.0
    return q * s[:, None]


def _qmul(a, b):
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def _conj(q):
    return q * np.array([1.0, -1.0, -1.0, -1.0])


def darboux(q, seg_len):
    """u_j = (2 / lbar_j) vec(conj(q_j) q_{j+1}) for the joints j = 0 .. N-2."""
    q = np.asarray(q, dtype=np.float64)
    if len(q) < 2:
        return np.zeros((0, 3))
    lbar = 0.5 * (seg_len[:-1] + seg_len[1:])
    r = _qmul(_conj(q[:-1]), q[1:])
    return (2.0 / lbar)[:, None] * r[:, 1:]


def errors(spec, x0, got_a, got_b, ref_a, ref_b, k, seg_len=None, disp=None, length=None):
    """Metric values (normalised as in the module docstring) for one rod.  x0: initial
    positions; got_a/got_b, ref_a/ref_b: (x, v, q, w) of the GPU and the oracle k steps before
    the end and at the end.  For a piece of a rod (consecutive points and the frames between
    them): seg_len of the piece, and the whole rod's largest displacement and length."""
    seg_len = spec.seg_len if seg_len is None else seg_len
    L = float(np.sum(spec.seg_len)) if length is None else float(length)
    f = lambda a: np.asarray(a, dtype=np.float64)
    xa, qa = f(got_a[0]), f(got_a[2])
    xb, qb = f(got_b[0]), f(got_b[2])
    rxa, rqa = f(ref_a[0]), f(ref_a[2])
    rxb, rqb = f(ref_b[0]), f(ref_b[2])
    out = {}
    if disp is None:
        disp = float(np.linalg.norm(rxb - f(x0), axis=1).max())
    disp = max(disp, 1e-3 * L)
    out["x"] = float(np.abs(xb - rxb).max()) / disp
    out["tip"] = float(np.linalg.norm(xb[-1] - rxb[-1])) / L
    out["q"] = float(np.abs(_qalign(qb, rqb) - rqb).max())
    u, ru = darboux(qb, seg_len), darboux(rqb, seg_len)
    out["u"] = float(np.abs(u - ru).max() / max(np.abs(ru).max(), 1.0 / L)) if len(ru) else 0.0
    dtk = k * spec.dt
    vb, rvb = (xb - xa) / dtk, (rxb - rxa) / dtk
    out["vbar"] = float(np.abs(vb - rvb).max() / max(np.abs(rvb).max(), 1e-3 * L / dtk))
    wr = lambda p, q: 2.0 * _qmul(_conj(p), _qalign(q, p))[:, 1:] / dtk
    wb, rwb = wr(qa, qb), wr(rqa, rqb)
    out["wbar"] = float(np.abs(wb - rwb).max() / max(np.abs(rwb).max(), 1e-3 / dtk))
    out["unit"] = float(np.abs(np.linalg.norm(qb, axis=1) - 1).max())
    return out


def worst(all_errs):
    """Largest value of each metric over several rods."""
    keys = all_errs[0].keys()
    return {k: max(e[k] for e in all_errs) for k in keys}


def violations(errs, tol=None):
    """Metrics above their bars (the unit-norm check only applies to FP32 results)."""
    tol = TOL if tol is None else tol
    return {k: v for k, v in errs.items() if k in tol and v > tol[k]}


def check_window(gpu, ref, rods, k, label, tol, say=print):
    """Whole-state comparison of every rod against the bars tol.  gpu: (states k steps before
    the end, states at the end), each a list of (x, v, q, w); ref: the same as oracle states.
    Returns the worst values; raises AssertionError naming the quantities above their bars."""
    errs = []
    for r, (spec, st) in enumerate(rods):
        o = lambda s: (s.x, s.v, s.q, s.w)
        e = errors(spec, st.x, gpu[0][r], gpu[1][r], o(ref[0][r]), o(ref[1][r]), k)
        assert all(np.isfinite(a).all() for a in gpu[1][r])
        say("%s rod %d N=%d: %s" % (label, r, spec.n, fmt(e)))
        errs.append(e)
    w = worst(errs)
    bars = TOL if tol is None else tol
    share = max(v / bars[m] for m, v in w.items() if m in bars)
    say("%s: largest share of a bar used %.2f" % (label, share))
    bad = violations(w, tol)
    assert not bad, "%s: above the bars: %s" % (label, bad)
    return w


def floor_bars(floor):
    """Bars of a window whose FP32 floor was measured live: max(base bar, FLOOR_FACTOR x
    floor) per quantity."""
    return {m: max(TOL[m], FLOOR_FACTOR * floor.get(m, 0.0)) for m in TOL}


def fmt(errs):
    return " ".join("%s %.2e" % (k, v) for k, v in errs.items())
