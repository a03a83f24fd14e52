"""GPU parity of internal friction (Sec. 2.1: the CoRdE model's dissipation terms damping
relative motion, translational and angular; Kelvin-Voigt reading) against the FP64 oracle.
Tolerance from the method's target: every point within 1e-4 x rod length after the run."""
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


def _curved(n, inext, td_over_dt, seed=6):
    """A curved, twisted clamped rod released under gravity, internal friction tau_d a multiple
    of the stable dt (the dashpots then take part in the stability rule)."""
    rng = np.random.default_rng(seed)
    x, q = W.curved_rod(n, 1.0 / n, rng, 0.05, twist_sigma=0.05)
    spec, _ = W.straight_rod(n, inextensible=inext, dt=1e-5)
    spec = spec.replace(seg_len=np.linalg.norm(np.diff(x, axis=0), axis=1), clamp_x0=tuple(x[0]),
                        clamp_q0=tuple(q[0]))
    dt0 = R.stable_dt(spec)
    spec = spec.replace(damp_int=td_over_dt * dt0)
    spec = spec.replace(dt=R.stable_dt(spec))
    st = W.RodState(x=x, v=np.zeros_like(x), q=q, w=np.zeros((n, 3)))
    return spec, st


def _gpu(specs_states, n_steps, spl=10):
    b = R.RodBatch([s for s, _ in specs_states])
    b.set_state_rods([st for _, st in specs_states])
    b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()
    info = b.buckets()
    b.close()
    return out, info


@pytest.mark.parametrize("inext", [False, True])
@pytest.mark.parametrize("n", [64, 700])
def test_damped_rod_vs_oracle(inext, n):
    spec, st = _curved(n, inext, 20.0)
    n_steps = 600
    (x, v, q, w), = _gpu([(spec, st)], n_steps)[0]
    ref, _ = O.Rod(spec).rollout(PM.fp32_input(st), n_steps)
    L = float(np.sum(spec.seg_len))
    ex = float(np.abs(x - ref.x).max())
    _say("%s N=%d tau_d %.2e dt %.2e: max|dx| %.2e (tol %.1e)"
         % ("inext" if inext else "ext", n, spec.damp_int, spec.dt, ex, 1e-4 * L))
    assert np.isfinite(x).all()
    assert ex <= 1e-4 * L
    # the friction acted: the undamped rod (same dt) ends elsewhere
    free, _ = O.Rod(spec.replace(damp_int=0.0)).rollout(PM.fp32_input(st), n_steps)
    assert np.abs(free.x - ref.x).max() > 10 * max(ex, 1e-6)


def test_damped_and_plain_rods_in_one_handle():
    """Damped and undamped rods of one shape step in separate buckets (kernel variants); each
    matches the oracle, and the undamped one is bitwise what it is alone."""
    a = _curved(64, True, 20.0, seed=7)
    b = _curved(64, True, 0.0, seed=8)
    b = (b[0].replace(dt=a[0].dt), b[1])
    out, info = _gpu([a, b], 300)
    _say("buckets %s" % info)
    assert len(info) == 2
    alone, _ = _gpu([b], 300)
    for u, v in zip(out[1], alone[0]):
        assert np.array_equal(u, v)
    ref, _ = O.Rod(a[0]).rollout(PM.fp32_input(a[1]), 300)
    assert np.abs(out[0][0] - ref.x).max() <= 1e-4


def test_internal_friction_arguments():
    spec, st = _curved(64, True, 20.0)
    other, ost = _curved(64, True, 0.0, seed=9)
    b = R.RodBatch([spec, other.replace(dt=spec.dt)])
    with pytest.raises(R.RodError):
        b.set_contact([[0, -1]], 0.1)
    with pytest.raises(R.RodError):
        b.set_bindings([[0, 5, 1, 5]], True)
    with pytest.raises(R.RodError):
        b.set_chunking(32)
    tris = W.tube_mesh(W.tube_centreline(), 0.01, 8)
    with pytest.raises(R.RodError):
        b.set_environment(tris, 0.1)
    b.set_state_rods([st, ost])
    with pytest.raises(R.RodError):
        b.adjoint_forward(10, 5)
    b.set_contact([[1, -1]], 0.1)   # the undamped rod may be grouped
    b.close()
    with pytest.raises(R.RodError):   # negative friction
        R.RodBatch([spec.replace(damp_int=-1.0)])
    long_spec, _ = W.straight_rod(3000, inextensible=True, dt=1e-6)
    with pytest.raises(R.RodError):   # would be chunked
        R.RodBatch([long_spec.replace(damp_int=1e-6)])
