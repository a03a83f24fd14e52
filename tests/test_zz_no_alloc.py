"""rod_step_state_noalloc (for callers that cannot allocate device memory) through the C ABI:
two calls in a row, the second on a smaller handle, each bitwise equal to rod_set_state +
rod_step + rod_get_state of the same handle from the same state; state arrays owned by the
caller; the refusals."""
import numpy as np
import pytest

from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print("[gpu-test] " + msg, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    yield


def _rods_big():
    """Several kernel-shape buckets: the two-instrument pair (driven clamps) and a batch of
    uneven rods with per-rod dt."""
    rods = list(W.config1().rods)
    wl = W.config3(n_rods=40, n_min=16, n_max=900)
    rods += [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods]
    return rods


def _rods_small():
    return list(W.config0().rods) + list(W.config1(n=64).rods)


def _reference(rods, n_steps, spl):
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    b.step(n_steps, spl)
    b.sync()
    out = b.get_state()
    b.close()
    return out


def _noalloc(rods, n_steps, spl):
    import torch
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])      # also sets the handle's time base (t0 = 0)
    host = b.get_state()
    dev = [torch.tensor(a, device="cuda") for a in host]
    before = b.get_state()
    b.step_state_noalloc(*dev, 0, n_steps, spl)
    b.sync()
    after = b.get_state()                          # the handle's own state is left alone
    nb = len(b.buckets())
    b.close()
    for u, v in zip(before, after):
        assert np.array_equal(u, v)
    return [t.cpu().numpy() for t in dev], nb


def test_noalloc_matches_rod_step_twice():
    big, small = _rods_big(), _rods_small()
    for label, rods, n_steps, spl in (("big", big, 300, 20), ("small", small, 120, 10)):
        ref = _reference(rods, n_steps, spl)
        got, nb = _noalloc(rods, n_steps, spl)
        _say("%s handle: %d rods in %d buckets, %d steps at %d per launch"
             % (label, len(rods), nb, n_steps, spl))
        for k, (u, v) in enumerate(zip(ref, got)):
            assert np.array_equal(u, v), (label, "xvqw"[k], float(np.abs(u - v).max()))


def test_noalloc_refusals():
    import torch
    rods = _rods_small()
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    dev = [torch.tensor(a, device="cuda") for a in b.get_state()]
    with pytest.raises(R.RodError, match="INVALID"):
        b.step_state_noalloc(*dev, 0, -1, 10)
    with pytest.raises(ValueError):
        b.step_state_noalloc(*[t.cpu() for t in dev], 0, 10, 10)   # host arrays
    b.step_state_noalloc(*dev, 0, 0, 10)                              # zero steps: nothing
    b.close()
    # more points than the scratch array holds (2^21): 1025 rods of 2048 elements
    n, rods_n = 2048, 1025
    spec, st = W.config2(n, False).rods[0]
    b = R.RodBatch([spec] * rods_n)
    tot_pts = rods_n * (n + 1)
    x = torch.zeros(3 * tot_pts, device="cuda")
    v = torch.zeros_like(x)
    q = torch.zeros(4 * rods_n * n, device="cuda")
    w = torch.zeros(3 * rods_n * n, device="cuda")
    with pytest.raises(R.RodError, match="at most"):
        b.step_state_noalloc(x, v, q, w, 0, 1, 1)
    b.close()
    # a handle with a chunked rod keeps per-handle chunk state: refused
    spec, st = W.config2(4096, True).rods[0]
    b = R.RodBatch([spec])
    b.set_state_rods([st])
    dev = [torch.tensor(a, device="cuda") for a in b.get_state()]
    with pytest.raises(R.RodError, match="UNSUPPORTED"):
        b.step_state_noalloc(*dev, 0, 10, 10)
    b.close()
