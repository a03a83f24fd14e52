"""GPU parity of the binding constraints (two rods bound by zero-length distance constraints,
stepped by one workgroup per pair) against the FP64 oracle's group step, from the same FP32
input.  The whole state (parity_metrics) is compared over the last 10 of the first 500 steps,
to bars derived from the configuration's FP32 floor; after 2000 steps every point is within
1e-4 x rod length (the method's target).  Between the two the free guidewire section buckles
(straight and compressed by the catheter's drive), in a direction that rounding decides, so
only positions are held to a bar there."""
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


def _gpu(rods, pairs, one_way, n_steps, spl=10, shape=None):
    b = R.RodBatch([s for s, _ in rods])
    if shape is not None:
        b.set_tuning(shape[0], shape[1], spl)
    if pairs is not None:
        b.set_bindings(pairs, one_way)
    b.set_state_rods([st for _, st in rods])
    b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()
    info = b.buckets()
    b.close()
    return out, info


@pytest.mark.parametrize("one_way", [True, False])
def test_catheter_guidewire_vs_oracle(one_way):
    case = parity_cases.bound_pair(one_way)
    pairs = case.bind[0]
    n, k, n_long = case.n_steps, case.window, 2000
    _say("c5 %s: 2x512 bound by %d pairs, %d + %d steps at 10 per launch"
         % ("one-way" if one_way else "two-way", len(pairs), n, n_long - n))
    b = R.RodBatch([s for s, _ in case.rods])
    case.setup(b)
    assert b.buckets() == [(4, 2, 2, 0.0)]
    b.set_state_rods([st for _, st in case.rods])
    b.step(n - k, 10)
    ga = b.get_state_rods()
    b.step(k, 10)
    gb = b.get_state_rods()
    b.step(n_long - n, 10)
    b.sync()
    gpu = b.get_state_rods()
    b.close()
    ra, rb, _ = parity_cases.group_window(O, case, n, k)
    PM.check_window((ga, gb), (ra, rb), case.rods, k, "c5-%d" % n, PM.BARS[case.bars], _say)
    ref, _ = parity_cases.group_run(O, case, n_long - n, states=rb, t0=n * case.rods[0][0].dt)
    for (x, v, q, w), o, (s, _) in zip(gpu, ref, case.rods):
        L = float(np.sum(s.seg_len))
        ex = float(np.abs(x - o.x).max())
        tip = float(np.linalg.norm(x[-1] - o.x[-1]))
        _say("  N=%d after %d: max|dx| %.2e tip %.2e (tol %.1e), |q|-1 %.1e" % (
            s.n, n_long, ex, tip, 1e-4 * L, np.abs(np.linalg.norm(q.astype(np.float64), axis=1) - 1).max()))
        assert np.isfinite(x).all() and np.isfinite(v).all()
        assert ex <= 1e-4 * L and tip <= 1e-4 * L
    # bound points coincide at the end of every step (binding is the last constraint)
    gap = np.abs(gpu[1][0][pairs[:, 1]] - gpu[0][0][pairs[:, 3]]).max()
    _say("  bound-point gap %.2e m" % gap)
    assert gap <= 1e-6
    # and they actually moved the rods: against the unbound run
    free, _ = _gpu(case.rods, None, one_way, n_long)
    moved = max(np.abs(gpu[r][0] - free[r][0]).max() for r in (0, 1))
    _say("  largest displacement from the unbound run %.2e m" % moved)
    assert moved > 1e-6


def test_one_way_master_is_bitwise_alone():
    """Variant 1: the master rod in the pair kernel evolves exactly as in the single-rod kernel
    (its arithmetic does not depend on the kernel shape or on the bound partner)."""
    wl, pairs = W.config5(True)
    gpu, _ = _gpu(wl.rods, pairs, True, 300)
    alone, _ = _gpu([wl.rods[0]], None, True, 300, shape=(4, 2))
    for u, v in zip(gpu[0], alone[0]):
        assert np.array_equal(u, v)
    assert np.abs(gpu[1][0] - _gpu([wl.rods[1]], None, True, 300)[0][0][0]).max() > 0


def test_cleared_bindings_step_independently():
    wl, pairs = W.config5(False)
    b = R.RodBatch([s for s, _ in wl.rods])
    b.set_bindings(pairs, False)
    assert b.buckets() == [(4, 2, 2, 0.0)]
    b.set_bindings([], False)
    assert b.buckets() == [(4, 2, 2, 0.0)] or len(b.buckets()) == 1
    b.set_state_rods([st for _, st in wl.rods])
    b.step(200, 10)
    got = b.get_state_rods()
    b.close()
    ref, _ = _gpu(wl.rods, None, False, 200)
    for a, c in zip(got, ref):
        for u, v in zip(a, c):
            assert np.array_equal(u, v)


def test_bound_pair_beside_other_rods():
    """A handle with a bound pair and unbound rods: the pair and the buckets step together,
    each as it would alone (whole state over the last 10 of 500 steps: the pair against the
    group step, the other rods one by one)."""
    case = parity_cases.bound_pair(False)
    extra = W.config0().rods + W.config2(700, True).rods
    rods = case.rods + extra
    b = R.RodBatch([s for s, _ in rods])
    case.setup(b)
    info = b.buckets()
    _say("mixed handle buckets %s" % info)
    assert (4, 2, 2, 0.0) in info
    b.set_state_rods([st for _, st in rods])
    b.step(490, 10)
    ga = b.get_state_rods()
    b.step(10, 10)
    gb = b.get_state_rods()
    b.close()
    ra, rb, _ = parity_cases.group_window(O, case, 500, 10)
    PM.check_window((ga[:2], gb[:2]), (ra, rb), case.rods, 10, "pair", PM.BARS["c5"], _say)
    oa = [O.Rod(s).rollout(st, 490)[0] for s, st in PM.fp32_rods(extra)]
    ob = [O.Rod(s).rollout(a, 10, t0=490 * s.dt)[0] for (s, _), a in zip(extra, oa)]
    PM.check_window((ga[2:], gb[2:]), (oa, ob), extra, 10, "unbound", PM.TOL, _say)


def test_binding_arguments():
    wl, pairs = W.config5(True)
    rods = wl.rods + W.config0().rods
    b = R.RodBatch([s for s, _ in rods])
    bad = [
        [[0, 0, 1, 5]],               # base point
        [[0, 513, 1, 5]],             # past the end
        [[0, 5, 0, 6]],               # same rod
        [[0, 5, 1, 5], [0, 5, 1, 6]],  # a point twice
        [[0, 5, 1, 5], [0, 6, 2, 6]],  # a rod bound to two others
        [[2, 5, 1, 5]],               # extensible rod
    ]
    for p in bad:
        with pytest.raises(R.RodError):
            b.set_bindings(p, False)
    with pytest.raises(R.RodError):   # one-way pairs naming both rods as master
        b.set_bindings([[0, 5, 1, 5], [1, 6, 0, 6]], True)
    b.set_bindings(pairs, True)
    b.set_state_rods([st for _, st in rods])
    with pytest.raises(R.RodError):
        b.adjoint_forward(10, 5)
    b.close()
