"""GPU parity of sphere contact (between two rods and within one rod, Coulomb friction) against
the FP64 oracle's group step.  Tolerance from the method's target: every point within
1e-4 x rod length after the run."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
import parity_metrics as PM

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.init()
    yield


def _crossing():
    wl = W.config6()
    dt = min(R.stable_dt(s) for s, _ in wl.rods)
    return [(s.replace(dt=dt), st) for s, st in wl.rods]


def _gpu(rods, sets, mu, n_steps, spl=10):
    b = R.RodBatch([s for s, _ in rods])
    if sets is not None:
        b.set_contact(sets, mu)
    b.set_state_rods([st for _, st in rods])
    b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()
    info = b.buckets()
    b.close()
    return out, info


def _compare(gpu, ref, rods, label):
    for (x, v, q, w), o, (s, _) in zip(gpu, ref, rods):
        L = float(np.sum(s.seg_len))
        ex = float(np.abs(x - o.x).max())
        _say("  %s N=%d: max|dx| %.2e (tol %.1e), |q|-1 %.1e" % (
            label, s.n, ex, 1e-4 * L, np.abs(np.linalg.norm(q.astype(np.float64), axis=1) - 1).max()))
        assert np.isfinite(x).all() and np.isfinite(v).all()
        assert ex <= 1e-4 * L


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_crossing_rods_vs_oracle(mu):
    rods = _crossing()
    n_steps = 2000
    _say("c6 crossing rods 2x128, mu %.1f, %d steps at 10 per launch" % (mu, n_steps))
    gpu, info = _gpu(rods, [[0, 1]], mu, n_steps)
    _say("buckets %s" % info)
    assert info == [(1, 2, 2, 0.0)]
    ref, most = O.rollout_group([s for s, _ in rods], [PM.fp32_input(st) for _, st in rods], n_steps, mu=mu)
    assert most >= 1
    _compare(gpu, ref, rods, "c6")
    # the falling rod rests on the bar: their middles a contact distance apart, not through
    gap = gpu[1][0][64, 2] - gpu[0][0][64, 2]
    _say("  middle-point gap %.5f m (contact distance 0.02)" % gap)
    assert gap >= 0.98 * 0.02


def coiled(n=48, turns=2, L=1.0, r=0.01, rise=0.5):
    """Two flat turns of a circle with a slight helical rise (the second turn rise x 2r above
    the first); the rest shape is this shape (intrinsic curvature from the oracle)."""
    R_ = L / (2 * np.pi * turns)
    s = np.linspace(0.0, L, n + 1)
    x = np.stack([R_ * np.sin(s / R_), R_ * (1 - np.cos(s / R_)), rise * 2 * r * s / (L / turns)], 1)
    q = W.frames_from_polyline(x)
    spec, st = W.straight_rod(n, L=L, radius=r, inextensible=True, dt=1e-5, gravity=(0, 0, 0),
                              damp=5.0)
    rod = O.Rod(spec)
    u_hat = np.array([rod.darboux(q, j) for j in range(n - 1)])
    lens = np.linalg.norm(x[1:] - x[:-1], axis=1)
    spec = spec.replace(u_hat=u_hat, seg_len=lens, clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    spec = spec.replace(dt=R.stable_dt(spec))
    st = st.copy()
    st.x, st.q = x, q
    return spec, st


def test_coiled_rod_self_contact_vs_oracle():
    """A single rod whose second turn lies on its first: self-contact pushes the turns apart."""
    spec, st = coiled()
    gpu, info = _gpu([(spec, st)], [[0, -1]], 0.2, 200)
    _say("coiled rod, self contact, 200 steps; buckets %s" % info)
    assert info == [(1, 2, 1, 0.0)]
    ref, most = O.rollout_group([spec], [PM.fp32_input(st)], 200, mu=0.2)
    assert most >= 1
    _compare(gpu, ref, [(spec, st)], "coiled")
    x = gpu[0][0]
    skip = O.self_skip(spec)
    closest = min(np.linalg.norm(x[i] - x[j]) for i in range(1, 49) for j in range(i + skip + 1, 49))
    _say("  closest non-neighbour points %.5f (contact distance 0.02)" % closest)
    assert closest >= 0.98 * 0.02


def test_contact_lists_across_launches_and_new_states():
    """The candidate lists are kept between launches and rebuilt only when points have moved;
    the contacts found do not depend on when that happens: 1, 7 or 100 steps per launch give
    bitwise the same states, and so does a handle that ran on and then got its state reset."""
    rods = _crossing()
    outs = [_gpu(rods, [[0, 1]], 0.3, 2000, spl=k)[0] for k in (1, 7, 100)]
    b = R.RodBatch([s for s, _ in rods])
    b.set_contact([[0, 1]], 0.3)
    b.set_state_rods([st for _, st in rods])
    b.step(1300, 10)
    b.set_state_rods([st for _, st in rods])
    b.step(2000, 10)
    b.sync()
    outs.append(b.get_state_rods())
    b.close()
    ref, most = O.rollout_group([s for s, _ in rods], [PM.fp32_input(st) for _, st in rods], 2000, mu=0.3)
    _say("crossing rods, 2000 steps at 1 / 7 / 100 per launch and after a reset; contacts %d" % most)
    assert most >= 1
    for o in outs[1:]:
        for a, c in zip(o, outs[0]):
            for u, v in zip(a, c):
                assert np.array_equal(u, v)
    _compare(outs[0], ref, rods, "c6")


def test_dense_side_by_side_contact_vs_oracle():
    """Two parallel rods whose elements are much shorter than their radius, one pressed
    sideways onto the other: every point near the other rod has more candidate partners (pairs
    within contact distance + margin) than a list holds, so each list build falls back to the
    exact contacts, which stay few."""
    n, r = 64, 0.01
    L = n * 0.08 * r
    a, sa = W.straight_rod(n, L=L, radius=r, young=1e7, inextensible=True, gravity=(0, 0, 0),
                           damp=0.5)
    b, sb = W.straight_rod(n, L=L, radius=r, young=1e6, inextensible=True,
                           gravity=(0, -9.81, 0), damp=0.5)
    off = np.array([0.0, 1.99 * r, 0.0])
    sb = sb.copy()
    sb.x = sb.x + off
    b = b.replace(clamp_x0=tuple(np.asarray(b.clamp_x0) + off))
    dt = min(R.stable_dt(a), R.stable_dt(b))
    rods = [(a.replace(dt=dt), sa), (b.replace(dt=dt), sb)]
    n_steps = 400
    gpu, info = _gpu(rods, [[0, 1]], 0.2, n_steps)
    ref, most = O.rollout_group([s for s, _ in rods], [PM.fp32_input(st) for _, st in rods], n_steps, mu=0.2)
    _say("side by side 2x%d, l = 0.08 r, %d steps: most contacts of a point %d" % (n, n_steps, most))
    assert 1 <= most <= 8
    _compare(gpu, ref, rods, "side by side")


def _unequal(gap=1e-3):
    """A 300-element bar along x (1 m, no gravity) and a 60-element rod along y (0.5 m) that
    falls across its middle from gap above; both radius 4 mm, inextensible, static clamps."""
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
    dt = min(R.stable_dt(s) for s, _ in out)
    return [(s.replace(dt=dt), st) for s, st in out]


def test_rods_of_different_lengths_vs_oracle():
    """Contact between a 300-element and a 60-element rod (one workgroup of two 4 x 2 halves,
    the short rod's half mostly idle)."""
    rods = _unequal()
    n_steps = 1500
    gpu, info = _gpu(rods, [[0, 1]], 0.2, n_steps)
    ref, most = O.rollout_group([s for s, _ in rods], [PM.fp32_input(st) for _, st in rods], n_steps, mu=0.2)
    _say("300 + 60 elements crossing, %d steps: buckets %s, contacts %d" % (n_steps, info, most))
    assert info == [(4, 2, 2, 0.0)]
    assert most >= 1
    _compare(gpu, ref, rods, "unequal")


def test_cleared_contact_steps_plainly():
    rods = _crossing()
    b = R.RodBatch([s for s, _ in rods])
    b.set_contact([[0, 1]], 0.3)
    b.set_contact([], 0.3)
    b.set_state_rods([st for _, st in rods])
    b.step(100, 10)
    got = b.get_state_rods()
    b.close()
    ref, _ = _gpu(rods, None, 0.0, 100)
    for a, c in zip(got, ref):
        for u, v in zip(a, c):
            assert np.array_equal(u, v)


def test_contact_arguments():
    rods = _crossing() + W.config0().rods
    b = R.RodBatch([s for s, _ in rods])
    for sets, mu in (([[0, 0]], 0.1), ([[0, 1], [1, -1]], 0.1), ([[0, 5]], 0.1),
                     ([[0, 1]], -1.0), ([[2, -1]], 0.1)):
        with pytest.raises(R.RodError):
            b.set_contact(sets, mu)
    b.set_contact([[0, 1]], 0.1)
    b.set_state_rods([st for _, st in rods])
    with pytest.raises(R.RodError):
        b.adjoint_forward(10, 5)
    b.close()
