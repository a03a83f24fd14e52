"""GPU parity of internal friction (Sec. 2.1: the CoRdE model's dissipation terms damping
relative motion, translational and angular; Kelvin-Voigt reading) against the FP64 oracle,
from the same FP32 input: the whole state (parity_metrics) over the last 10 steps of each run,
to bars from the configurations' FP32 floor; the tip within 1e-4 x rod length (the method's
target)."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
import parity_cases
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
    return parity_cases.damped(O, n, inext, td_over_dt, seed)


def _gpu(specs_states, n_steps, spl=10, window=0):
    """States after n_steps (and, with a window k, after n_steps - k), and the buckets."""
    b = R.RodBatch([s for s, _ in specs_states])
    b.set_state_rods([st for _, st in specs_states])
    before = None
    if window:
        b.step(n_steps - window, spl)
        before = b.get_state_rods()
        b.step(window, spl)
    else:
        b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()
    info = b.buckets()
    b.close()
    return (out, info) if not window else (before, out, info)


def _oracle_window(specs_states, n_steps, k):
    a = [O.Rod(s).rollout(PM.fp32_input(st), n_steps - k)[0] for s, st in specs_states]
    b = [O.Rod(s).rollout(sa, k, t0=(n_steps - k) * s.dt)[0] for (s, _), sa in zip(specs_states, a)]
    return a, b


@pytest.mark.parametrize("inext", [False, True])
@pytest.mark.parametrize("n", [64, 700])
def test_damped_rod_vs_oracle(inext, n):
    """Whole state over the last 10 of 600 steps against the oracle (bars from the
    configuration's FP32 floor); the tip within 1e-4 x rod length."""
    rod = _curved(n, inext, 20.0)
    spec = rod[0]
    n_steps, k = 600, 10
    ga, gb, _ = _gpu([rod], n_steps, window=k)
    ra, rb = _oracle_window([rod], n_steps, k)
    label = "%s N=%d tau_d %.2e dt %.2e" % ("inext" if inext else "ext", n, spec.damp_int, spec.dt)
    PM.check_window((ga, gb), (ra, rb), [rod], k, label, PM.BARS["damped"], _say)
    # the friction acted: the undamped rod (same dt) ends elsewhere
    free, _ = O.Rod(spec.replace(damp_int=0.0)).rollout(PM.fp32_input(rod[1]), n_steps)
    ex = float(np.abs(gb[0][0] - rb[0].x).max())
    assert np.abs(free.x - rb[0].x).max() > 10 * max(ex, 1e-6)


def test_damped_and_plain_rods_in_one_handle():
    """Damped and undamped rods of one shape step in separate buckets (kernel variants); each
    matches the oracle, and the undamped one is bitwise what it is alone."""
    a = _curved(64, True, 20.0, seed=7)
    b = _curved(64, True, 0.0, seed=8)
    b = (b[0].replace(dt=a[0].dt), b[1])
    ga, gb, info = _gpu([a, b], 300, window=10)
    _say("buckets %s" % info)
    assert len(info) == 2
    alone, _ = _gpu([b], 300)
    for u, v in zip(gb[1], alone[0]):
        assert np.array_equal(u, v)
    ra, rb = _oracle_window([a, b], 300, 10)
    PM.check_window((ga, gb), (ra, rb), [a, b], 10, "damped + plain", PM.BARS["damped"], _say)


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
