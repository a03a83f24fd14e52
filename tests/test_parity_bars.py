"""The GPU parity bars can fail: on each parity configuration, the FP64 oracle with one
coefficient of the method changed by 10 % (or one constraint iteration in ten dropped) is
compared with the unchanged oracle by the same whole-state metrics and bars as the GPU
(parity_metrics), and must break at least one bar wherever the table below says the
configuration covers that coefficient.  Every step of the method is covered somewhere:

  external forces (gravity, linear and angular damping, clamp drive)   Sec. 2.1, Fig. 5
  stretch / shear (K_s of eq. (2), K_p of eq. (8))                      eqs. (2), (8)
  bend / twist (K_1 = K_2, K_3 of eq. (3))                              eqs. (3), (5), (6)
  force integration (masses and inertias: the density)                  Sec. 2.1
  distance constraints (the number of constraint iterations)            Sec. 2.1
  velocity integration (the time step)                                  Sec. 2.1
  internal friction (the retardation time of the Kelvin-Voigt dashpots)  Sec. 2.1
  binding constraints (a tenth of the bound points released)           Sec. 3.4
  contact friction (the Coulomb coefficient)                            Sec. 2.3

The bound and touching configurations (parity_cases.group_cases) are held to the same rules:
their bars follow their FP32 floors, and they detect the changes listed for them.  So are the
restart windows of the environment-collision tests (10 steps from states along a run, bars
from each window's own floor).
"""
import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_2509_04277_amd import workloads as W
import parity_cases
import parity_metrics as PM


def _g(s, f):
    return s.replace(gravity=tuple(f * g for g in s.gravity))


# 10 % changes, each of one coefficient (K_s alone: E up, the other stiffnesses scaled back)
CHANGES = {
    "gravity": lambda s: _g(s, 1.1),
    "damp_lin": lambda s: s.replace(damp_lin=1.1 * s.damp_lin),
    "damp_ang": lambda s: s.replace(damp_ang=1.1 * s.damp_ang),
    "drive": lambda s: s.replace(clamp_amp=tuple(1.1 * a for a in s.clamp_amp),
                                 clamp_twist_amp=1.1 * s.clamp_twist_amp),
    "K_s": lambda s: s.replace(young=1.1 * s.young, kp_scale=s.kp_scale / 1.1,
                               bend_scale=s.bend_scale / 1.1, twist_scale=s.twist_scale / 1.1),
    "K_p": lambda s: s.replace(kp_scale=1.1 * s.kp_scale),
    "bend": lambda s: s.replace(bend_scale=1.1 * s.bend_scale),
    "twist": lambda s: s.replace(twist_scale=1.1 * s.twist_scale),
    "mass": lambda s: s.replace(density=1.1 * s.density),
    "n_iter": lambda s: s.replace(n_iter=s.n_iter - max(1, s.n_iter // 10)) if s.inextensible else s,
    "dt": lambda s: s.replace(dt=1.1 * s.dt),
    "damp_int": lambda s: s.replace(damp_int=1.1 * s.damp_int),
}

# changes of the group step's own arguments (the oracle's rollout_group keywords)
GROUP_CHANGES = {
    "bind": lambda kw: dict(kw, pairs=kw["pairs"][len(kw["pairs"]) // 10:]),
    "mu": lambda kw: dict(kw, mu=1.1 * kw["mu"]),
}

# configuration: (rods, steps, window, bar set, coefficients it must detect)
ALL = tuple(CHANGES)

# group configuration: coefficients it must detect
GROUP_MUST = {
    "c5-one": ("drive", "twist", "mass", "dt", "bind"),
    "c5-two": ("drive", "twist", "mass", "n_iter", "dt", "bind"),
}

# touching rods: checked in restart windows (parity_cases.TOUCHING_STOPS); the changes that
# must break the bars of at least one window
TOUCHING_MUST = {
    "c6-mu0": ("K_p", "bend", "mass", "dt"),
    "c6-mu0.3": ("K_p", "bend", "mass", "dt", "mu"),
    "coiled": ("K_p", "bend", "twist", "mass", "dt"),
    "side": ("K_p", "bend", "mass", "dt", "mu"),
    "unequal": ("K_p", "bend", "mass", "dt"),
}


def _configs(oracle):
    return {
        "c0": (W.config0().rods, 2000, 10, "c0",
               ("gravity", "K_s", "K_p", "bend", "twist", "mass", "dt")),
        "c0-swing": (W.config0(dt=1e-4).rods, 3000, 50, "c0-swing",
                     ("gravity", "damp_lin", "K_s", "K_p", "bend", "twist", "mass", "dt")),
        "c1-2000": (W.config1().rods, 2000, 10, "c1", ("twist", "mass", "n_iter", "dt", "drive")),
        "c1-full": (W.config1().rods, 20000, 10, "c1-full",
                    ("bend", "twist", "mass", "n_iter", "dt", "drive")),
        "edge": (parity_cases.edge_rods(oracle), 400, 37, "edge",
                 tuple(c for c in ALL if c != "damp_int")),   # (no internal friction there)
        "c2-4096": (W.config2(4096, True).rods + W.config2(4096, False).rods, 5000, 10, "c2", ()),
        "c0-300": (W.config0(n=64).rods, 300, 10, "c0", ()),
        "batch": (parity_cases.batch48(oracle), 150, 10, "batch", ()),
        "c3-sampled": (_c3_sample(oracle), 1000, 10, "c3", ()),
        "damped": ([parity_cases.damped(oracle, n, inext, 20.0) for n in (64, 700)
                    for inext in (False, True)], 600, 10, "damped",
                   ("gravity", "K_s", "K_p", "bend", "twist", "mass", "dt", "damp_int")),
    }


def _c3_sample(oracle):
    rods = parity_cases.with_rule_dt(oracle, W.config3().rods)
    return [rods[i] for i in parity_cases.c3_pick(rods)]


def _window(oracle, rods, n, k):
    """States k steps before the end and at the end (the rods on the oracle's threads)."""
    a = oracle.rollout_many_threads(rods, n - k)
    b = [oracle.Rod(s).rollout(sa, k, t0=(n - k) * s.dt)[0] for (s, _), sa in zip(rods, a)]
    return a, b


def _differs(a, b):
    return any(not np.array_equal(np.asarray(getattr(a, f.name), dtype=object),
                                  np.asarray(getattr(b, f.name), dtype=object))
               for f in dataclasses.fields(a))


def _t(st):
    return (st.x, st.v, st.q, st.w)


def _worst(rods, pa, pb, a, b, k):
    return PM.worst([PM.errors(s, st.x, _t(x), _t(y), _t(u), _t(v), k)
                     for (s, st), x, y, u, v in zip(rods, pa, pb, a, b)])


def test_every_step_is_covered(oracle):
    """Together the configurations cover every coefficient of CHANGES."""
    covered = set()
    for _, _, _, _, must in _configs(oracle).values():
        covered |= set(must)
    for must in list(GROUP_MUST.values()) + list(TOUCHING_MUST.values()):
        covered |= set(must)
    for _, _, must in ENV.values():
        covered |= set(must)
    assert covered == set(CHANGES) | set(GROUP_CHANGES)
    assert set(GROUP_MUST) | set(TOUCHING_MUST) == set(parity_cases.group_cases(oracle))


NAMES = ["c0", "c0-swing", "c1-2000", "c1-full", "edge", "damped"]


@pytest.mark.parametrize("name", NAMES)
def test_bars_fail_on_changed_coefficients(oracle, name):
    rods, n, k, bars, must = _configs(oracle)[name]
    rods = PM.fp32_rods(rods)
    a, b = _window(oracle, rods, n, k)
    same = _worst(rods, a, b, a, b, k)
    same.pop("unit")
    assert all(v == 0.0 for v in same.values())
    changed = []
    for coef in must:
        prods = [(CHANGES[coef](s), st) for s, st in rods]
        assert any(_differs(ps, s) for (ps, _), (s, _) in zip(prods, rods)), coef
        changed += prods
    pa = oracle.rollout_many_threads(changed, n - k)
    missed = []
    for i, coef in enumerate(must):
        sl = slice(i * len(rods), (i + 1) * len(rods))
        pb = [oracle.Rod(s).rollout(x, k, t0=(n - k) * s.dt)[0] for (s, _), x in zip(changed[sl], pa[sl])]
        w = _worst(rods, pa[sl], pb, a, b, k)
        w.pop("unit")   # an FP64 oracle keeps unit quaternions whatever its coefficients
        bad = PM.violations(w, PM.BARS[bars])
        print("%s, %s x1.1: %s -> above the bars: %s" % (name, coef, PM.fmt(w), sorted(bad)))
        if not bad:
            missed.append(coef)
    assert not missed, "%s: a 10 %% change of %s passes every bar" % (name, missed)


def _up2(v):
    """v rounded up to two significant digits."""
    e = math.floor(math.log10(v))
    return math.ceil(v / 10 ** (e - 1) - 1e-9) * 10 ** (e - 1)


@pytest.mark.parametrize("name", NAMES + ["c2-4096", "c0-300", "batch", "c3-sampled"])
def test_bars_follow_the_fp32_floor(oracle, name):
    """Each bar is max(base bar, FLOOR_FACTOR x the configuration's FP32 floor), the floor
    being the oracle against itself with v, q and w rounded to FP32 after every step."""
    rods, n, k, bars, _ = _configs(oracle)[name]
    rods = PM.fp32_rods(rods)
    a, b = _window(oracle, rods, n, k)
    def one(args):
        (s, st), sa, sb = args
        r = oracle.Rod(s)
        ra = r.rollout_rounded(st, n - k, 14)
        rb = r.rollout_rounded(ra, k, 14, t0=(n - k) * s.dt)
        return PM.errors(s, st.x, _t(ra), _t(rb), _t(sa), _t(sb), k)
    with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:   # ctypes drops the GIL
        fl = list(ex.map(one, zip(rods, a, b)))
    floor = PM.worst(fl)
    floor.pop("unit")
    print("%s: FP32 floor %s" % (name, PM.fmt(floor)))
    _check_bars(name, floor, PM.BARS[bars])


def _check_bars(name, floor, bars):
    """Each bar within 20 % of max(base bar, FLOOR_FACTOR x floor) rounded up to two digits
    (the floors move in their last digits between machines)."""
    for m, f in floor.items():
        want = max(PM.TOL[m], _up2(PM.FLOOR_FACTOR * f)) if f > 0 else PM.TOL[m]
        got = bars[m]
        assert 0.8 * want <= got <= 1.2 * want, (name, m, got, want)


def _group_worst(case, pa, pb, a, b):
    return PM.worst([PM.errors(s, st.x, _t(x), _t(y), _t(u), _t(v), case.window)
                     for (s, st), x, y, u, v in zip(case.rods, pa, pb, a, b)])


@pytest.mark.parametrize("name", sorted(GROUP_MUST))
def test_group_bars_fail_on_changed_coefficients(oracle, name):
    case = parity_cases.group_cases(oracle)[name]
    n, k = case.n_steps, case.window
    a, b, _ = parity_cases.group_window(oracle, case, n, k)
    specs = [s for s, _ in case.rods]
    missed = []
    for coef in GROUP_MUST[name]:
        if coef in CHANGES:
            cs = [CHANGES[coef](s) for s in specs]
            assert any(_differs(c, s) for c, s in zip(cs, specs)), coef
            pa, pb, _ = parity_cases.group_window(oracle, case, n, k, specs=cs)
        else:
            kw = GROUP_CHANGES[coef](dict(case.oracle_kw))
            pa, pb, _ = parity_cases.group_window(oracle, case, n, k, **kw)
        w = _group_worst(case, pa, pb, a, b)
        w.pop("unit")
        bad = PM.violations(w, PM.BARS[case.bars])
        print("%s, %s changed: %s -> above the bars: %s" % (name, coef, PM.fmt(w), sorted(bad)))
        if not bad:
            missed.append(coef)
    assert not missed, "%s: a change of %s passes every bar" % (name, missed)


@pytest.mark.parametrize("bars", ["c5"])
def test_group_bars_follow_the_fp32_floor(oracle, bars):
    """As test_bars_follow_the_fp32_floor, for the bound and touching configurations (every
    rod of the group rounded after every group step); a bar set that several configurations
    share follows the largest of their floors."""
    cases = [c for c in parity_cases.group_cases(oracle).values() if c.bars == bars]
    assert cases
    fl = []
    for case in cases:
        n, k = case.n_steps, case.window
        a, b, _ = parity_cases.group_window(oracle, case, n, k)
        ra, rb, _ = parity_cases.group_window(oracle, case, n, k, round_mask=14)
        fl.append(_group_worst(case, ra, rb, a, b))
    floor = PM.worst(fl)
    floor.pop("unit")
    print("%s: FP32 floor %s" % (bars, PM.fmt(floor)))
    _check_bars(bars, floor, PM.BARS[bars])


# environment collision: restart steps along the run, and the changes those windows detect
ENV = {
    "tube-0.0": (lambda o: parity_cases.tube(o, 0.0), (400, 600, 800, 1000, 1190),
                 ("gravity", "K_p", "bend", "twist", "mass", "dt")),
    "tube-0.3": (lambda o: parity_cases.tube(o, 0.3), (400, 600, 800, 1000, 1190),
                 ("gravity", "K_p", "bend", "twist", "mass", "dt")),
    "floor-inext": (lambda o: parity_cases.on_floor(o, True), (200, 500, 1000, 1490),
                    ("gravity", "K_p", "bend", "mass", "n_iter", "dt")),
    "floor-ext": (lambda o: parity_cases.on_floor(o, False), (200, 500, 1000, 1490),
                  ("gravity", "K_s", "K_p", "bend", "mass", "dt")),
}


@pytest.mark.parametrize("name", sorted(ENV))
def test_env_restart_bars_fail_on_changed_coefficients(oracle, name):
    make, stops, must = ENV[name]
    case = make(oracle)
    spec, st0 = case.rods[0]
    states, st, prev = [], None, 0
    for s in stops:
        st, _ = parity_cases.env_run(oracle, case, s - prev, state=st, t0=prev * spec.dt)
        prev = s
        states.append(st)
    base = parity_cases.env_restarts(oracle, case, states, stops)
    bars = [PM.floor_bars(parity_cases.window_floor(spec, st0.x, S, b, pert, 10, PM.errors))
            for S, b, pert in base]
    missed = []
    for coef in must:
        if coef == "mu":
            ch = parity_cases.env_changed(case, mu=1.1 * case.mu)
        else:
            ns = CHANGES[coef](spec)
            assert _differs(ns, spec), coef
            ch = parity_cases.env_changed(case, spec=ns)
        hit = []
        for (S, b, _), (_, pb, _), bb, s in zip(base, parity_cases.env_restarts(oracle, ch, states, stops),
                                                 bars, stops):
            e = PM.errors(spec, st0.x, _t(S), _t(pb), _t(S), _t(b), 10)
            e.pop("unit")
            if PM.violations(e, bb):
                hit.append(s)
        print("%s, %s changed: windows above their bars start at %s" % (name, coef, hit))
        if not hit:
            missed.append(coef)
    assert not missed, "%s: a change of %s passes every window" % (name, missed)


@pytest.mark.parametrize("name", sorted(TOUCHING_MUST))
def test_touching_restart_bars_fail_on_changed_coefficients(oracle, name):
    """As the environment restart windows: from the oracle's states at the configuration's
    restart steps, a changed coefficient must break the bars of some window."""
    case = parity_cases.group_cases(oracle)[name]
    stops = parity_cases.TOUCHING_STOPS[name]
    dt = case.rods[0][0].dt
    states, st, prev = [], None, 0
    for s in stops:
        st, _ = parity_cases.group_run(oracle, case, s - prev, states=st, t0=prev * dt)
        prev = s
        states.append(st)
    x0s = [st0.x for _, st0 in case.rods]
    base = parity_cases.group_restarts(oracle, case, states, stops)
    bars = [PM.floor_bars(parity_cases.group_floor(case, x0s, a, b, pert, 10, PM.errors))
            for a, b, pert in base]
    specs = [sp for sp, _ in case.rods]
    missed = []
    for coef in TOUCHING_MUST[name]:
        hit = []
        for (a, b, _), bb, s in zip(base, bars, stops):
            if coef in CHANGES:
                cs = [CHANGES[coef](sp) for sp in specs]
                assert any(_differs(c, sp) for c, sp in zip(cs, specs)), coef
                pb, _ = parity_cases.group_run(oracle, case, 10, states=a, t0=s * dt, specs=cs)
            else:
                kw = GROUP_CHANGES[coef](dict(case.oracle_kw))
                pb, _ = parity_cases.group_run(oracle, case, 10, states=a, t0=s * dt, **kw)
            w = PM.worst([PM.errors(sp, x0, _t(u), _t(v), _t(u), _t(r), 10)
                          for sp, x0, u, v, r in zip(specs, x0s, a, pb, b)])
            w.pop("unit")
            if PM.violations(w, bb):
                hit.append(s)
        print("%s, %s changed: windows above their bars start at %s" % (name, coef, hit))
        if not hit:
            missed.append(coef)
    assert not missed, "%s: a change of %s passes every window" % (name, missed)
