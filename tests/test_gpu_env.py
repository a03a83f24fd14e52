"""GPU parity of environment collision (Sec. 2.2 "Collisions": AABB tree broad phase,
sphere-triangle narrow phase, depth-weighted response normal; contact impulses with Coulomb
friction) against the FP64 oracle, which checks every triangle by brute force; both from the
same FP32 input and mesh.  A run against the mesh is ill-conditioned once points touch it
(contacts switch on and off, between triangles, between stick and slip), so:
  - along the run, from the GPU's state at several steps, 10 more steps on the GPU and on the
    oracle are compared as a whole state (parity_metrics), to bars of max(base bar, 10 x that
    window's FP32 floor: how far the oracle moves from itself over the window with v, q and w
    rounded after every step, or from a start moved by 2^-22 relative);
  - at the end of the run every point is within the method's target, 1e-4 x rod length, or 10x
    how far the oracle's own positions move when its state is rounded to FP32 after every
    step, whichever is larger."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
import parity_cases as PC
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


def _tube(n=64):
    wl, tris = W.config7(n=n)
    spec, st = wl.rods[0]
    return spec.replace(dt=R.stable_dt(spec)), st, tris


def _gpu(spec, st, n_steps, tris=None, mu=0.0, spl=10, haptic=False):
    b = R.RodBatch([spec])
    if tris is not None:
        b.set_environment(tris, mu)
    if haptic:
        b.haptic_attach(0, 5)
    b.set_state_rods([st])
    b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()[0]
    info = b.environment_info()
    b.close()
    return out, info


def _state(t):
    x, v, q, w = (np.asarray(a, dtype=np.float64) for a in t)
    return W.RodState(x=x, v=v, q=q, w=w)


def _run_with_stops(case, stops, spl=10):
    """The case's run on the GPU, its state at each stop and at the end; the tree's size."""
    spec, st = case.rods[0]
    b = R.RodBatch([spec])
    b.set_environment(case.tris, case.mu)
    b.set_state_rods([st])
    got, done = [], 0
    for s in list(stops) + [case.n_steps]:
        b.step(s - done, spl)
        done = s
        got.append(b.get_state_rods()[0])
    info = b.environment_info()
    b.close()
    return got[:-1], got[-1], info


def _restart_windows(case, starts, stops, label, k=10):
    """From each GPU state, k steps on the GPU (a handle set to that state) and on the oracle,
    whole state against bars from that window's FP32 floor."""
    spec, st0 = case.rods[0]
    b = R.RodBatch([spec])
    b.set_environment(case.tris, case.mu)
    gpu = []
    for S, s in zip(starts, stops):
        b.set_state_rods([_state(S)], t0=s * spec.dt)
        b.step(k, k)
        gpu.append(b.get_state_rods()[0])
    b.close()
    refs = PC.env_restarts(O, case, [_state(S) for S in starts], stops, k)
    for g, (S, ref, pert), s in zip(gpu, refs, stops):
        t = lambda u: (u.x, u.v, u.q, u.w)
        bars = PM.floor_bars(PC.window_floor(spec, st0.x, S, ref, pert, k, PM.errors))
        PM.check_window(([t(S)], [g]), ([S], [ref]), case.rods, k, "%s from step %d" % (label, s),
                        bars, _say)


def _fp32_storage_dev(case, ref):
    """max |dx| between the oracle's run and the same run with v, q and w rounded to FP32
    after every step."""
    r, _ = PC.env_run(O, case, case.n_steps, round_mask=14)
    return float(np.abs(r.x - ref.x).max())


@pytest.mark.parametrize("mu", [0.0, 0.3])
def test_rod_in_bent_tube_vs_oracle(mu):
    case = PC.tube(O, mu)
    stops = (400, 600, 800, 1000, 1190)
    _say("c7: 64-element rod in a bent tube of %d triangles, mu %.1f, %d steps"
         % (len(case.tris), mu, case.n_steps))
    starts, (x, v, q, w), info = _run_with_stops(case, stops)
    _say("  tree: %d nodes, %d triangles" % info)
    assert info[1] == len(case.tris) and info[0] >= len(case.tris) // 2
    ref, most = PC.env_run(O, case, case.n_steps)
    ex = float(np.abs(x - ref.x).max())
    tol = max(1e-4, PM.FLOOR_FACTOR * _fp32_storage_dev(case, ref))
    _say("  max|dx| %.2e (tol %.2e), colliding points (oracle, most) %d" % (ex, tol, most))
    assert most >= 3 and np.isfinite(x).all()
    assert ex <= tol
    cen = W.tube_centreline(ds=0.002)
    off_axis = np.linalg.norm(x[:, None, :] - cen[None, :, :], axis=2).min(axis=1).max()
    _say("  largest distance from the tube's axis %.4f (tube radius 0.01)" % off_axis)
    assert off_axis <= 0.01
    _restart_windows(case, starts, stops, "c7 mu %.1f" % mu)


@pytest.mark.parametrize("inext", [True, False])
def test_rod_falls_onto_a_floor_vs_oracle(inext):
    """A clamped rod sags onto a floor just below it and slides on it with friction."""
    case = PC.on_floor(O, inext)
    stops = (200, 500, 1000, 1490)
    starts, (x, v, q, w), _ = _run_with_stops(case, stops)
    ref, most = PC.env_run(O, case, case.n_steps)
    ex = float(np.abs(x - ref.x).max())
    tol = max(1e-4 * 0.5, PM.FLOOR_FACTOR * _fp32_storage_dev(case, ref))
    _say("floor, %s: max|dx| %.2e (tol %.2e), lowest point %.5f (floor + radius %.5f), colliding %d"
         % ("inextensible" if inext else "extensible", ex, tol, x[1:, 2].min(), -0.02 + 0.01, most))
    assert most >= 5
    assert ex <= tol
    assert x[1:, 2].min() >= -0.02 + 0.01 - 2e-3   # resting on it, not through it
    _restart_windows(case, starts, stops, "floor %s" % ("inext" if inext else "ext"))


def test_out_of_reach_mesh_is_the_plain_step():
    """A mesh no point reaches: the collision variant steps bitwise as the plain kernel, and a
    removed mesh gives the plain kernel back."""
    spec, st, tris = _tube()
    far = tris + np.array([0.0, 0.0, 50.0])
    plain, _ = _gpu(spec, st, 200)
    got, _ = _gpu(spec, st, 200, far, 0.3)
    for u, v in zip(plain, got):
        assert np.array_equal(u, v)
    b = R.RodBatch([spec])
    b.set_environment(tris, 0.3)
    b.set_environment([], 0.3)
    assert b.environment_info() == (0, 0)
    b.set_state_rods([st])
    b.step(200, 10)
    again = b.get_state_rods()[0]
    b.close()
    for u, v in zip(plain, again):
        assert np.array_equal(u, v)


def test_mailbox_and_environment_together():
    """The variant with both the mailbox and the collision code steps bitwise as the collision
    variant, and its force records stay finite."""
    spec, st, tris = _tube()
    a, _ = _gpu(spec, st, 600, tris, 0.3)
    b = R.RodBatch([spec])
    b.set_environment(tris, 0.3)
    b.haptic_attach(0, 5)
    b.set_state_rods([st])
    b.step(600, 10)
    b.sync()
    f, s, p = b.haptic_get_force(0)
    got = b.get_state_rods()[0]
    b.close()
    assert s == 600 and np.isfinite(f).all()
    for u, v in zip(a, got):
        assert np.array_equal(u, v)


def test_environment_arguments():
    spec, st, tris = _tube()
    other, ost = W.straight_rod(64, inextensible=True, dt=spec.dt)
    b = R.RodBatch([spec, other])
    for bad_t, bad_mu in ((tris, -1.0), (tris, float("nan")), (np.full((1, 3, 3), np.nan), 0.1)):
        with pytest.raises(R.RodError):
            b.set_environment(bad_t, bad_mu)
    b.set_environment(tris, 0.2)
    with pytest.raises(R.RodError):
        b.set_contact([[1, -1]], 0.1)
    with pytest.raises(R.RodError):
        b.set_chunking(32)
    b.set_state_rods([st, ost])
    with pytest.raises(R.RodError):
        b.adjoint_forward(10, 5)
    b.set_environment([], 0.2)
    b.set_contact([[1, -1]], 0.1)
    with pytest.raises(R.RodError):
        b.set_environment(tris, 0.2)   # grouped rods do not collide with the mesh
    b.close()
    # degenerate triangles are dropped
    b = R.RodBatch([spec])
    deg = np.concatenate([tris[:10], np.zeros((3, 3, 3))])
    b.set_environment(deg, 0.0)
    assert b.environment_info()[1] == 10
    b.close()
