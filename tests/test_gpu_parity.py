"""GPU parity: the HIP stepper (through the C ABI) against the FP64 oracle on the same seeded
inputs.  Every run is compared as a whole state (parity_metrics): positions (relative to how
far the rod moved, and the tip within 1e-4 x rod length, the method's target), frames,
Darboux vectors, and window-mean linear and angular velocities over the run's last steps;
quaternions unit to FP32 precision.  A CPU test (test_parity_bars) shows that a 10 % change of
each coefficient of the method breaks these bars on the configurations run here.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
import parity_cases
import parity_metrics as PM

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    print("[gpu-test] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert os.path.exists(R.LIB_PATH), "libcorde_rod.so must be built before the GPU tests"
    torch.cuda.init()
    yield


def run_gpu(rods, n_steps, spl, shape=None, t0=0.0):
    b = R.RodBatch([s for s, _ in rods])
    if shape is not None:
        b.set_tuning(shape[0], shape[1], spl)
    b.set_state_rods([st for _, st in rods], t0=t0)
    if n_steps:
        b.step(n_steps, spl)
    b.sync()
    out = b.get_state_rods()
    b.close()
    return out


def run_gpu_window(rods, n_steps, k, spl, shape=None):
    """States after n_steps - k and after n_steps steps (launches of spl steps; how a run is
    split into launches does not change its result)."""
    b = R.RodBatch([s for s, _ in rods])
    if shape is not None:
        b.set_tuning(shape[0], shape[1], spl)
    b.set_state_rods([st for _, st in rods])
    b.step(n_steps - k, spl)
    a = b.get_state_rods()
    b.step(k, spl)
    c = b.get_state_rods()
    b.close()
    return a, c


def run_oracle_window(oracle, rods, n_steps, k):
    a = [oracle.Rod(s).rollout(st, n_steps - k)[0] for s, st in PM.fp32_rods(rods)]
    c = [oracle.Rod(s).rollout(sa, k, t0=(n_steps - k) * s.dt)[0] for (s, _), sa in zip(rods, a)]
    return a, c


def compare_window(gpu, ref, rods, k, label, tol=None):
    """Whole-state comparison (parity_metrics) of every rod; returns the worst values."""
    return PM.check_window(gpu, ref, rods, k, label, tol, _say)


def test_c0_full_run(oracle):
    wl = W.config0()
    _say("c0 full: 1x64 extensible, %d steps, %d per launch" % (wl.n_steps, wl.steps_per_launch))
    gpu = run_gpu_window(wl.rods, wl.n_steps, 10, wl.steps_per_launch)
    ref = run_oracle_window(oracle, wl.rods, wl.n_steps, 10)
    compare_window(gpu, ref, wl.rods, 10, "c0", PM.BARS["c0"])


@pytest.mark.parametrize("shape", [(1, 1), (1, 2), (1, 4), (2, 1), (2, 2), (4, 1), (8, 1)])
def test_c0_every_kernel_shape(oracle, shape):
    wl = W.config0(dt=1e-4)
    _say("c0 dt=1e-4 (large swing), 3000 steps, shape waves=%d elems=%d" % shape)
    gpu = run_gpu_window(wl.rods, 3000, 50, 50, shape)
    ref = run_oracle_window(oracle, wl.rods, 3000, 50)
    compare_window(gpu, ref, wl.rods, 50, "c0-swing %s" % (shape,), PM.BARS["c0-swing"])


def test_c1_reduced_vs_oracle(oracle):
    wl = W.config1()
    _say("c1 2x512 inextensible, 2000 steps, 10 per launch, shape (4,2)")
    gpu = run_gpu_window(wl.rods, 2000, 10, 10, (4, 2))
    ref = run_oracle_window(oracle, wl.rods, 2000, 10)
    compare_window(gpu, ref, wl.rods, 10, "c1-2000", PM.BARS["c1"])


def test_c1_full_run_against_stored_oracle(oracle):
    """Full 20000-step run in the benchmark's launch configuration: the tip every 1000 steps and
    sample points against the stored FP64 oracle, and the whole state of the last 10 steps
    against a live oracle run."""
    g = json.load(open(os.path.join(HERE, "golden", "c1_oracle.json")))
    wl = W.config1()
    assert g["n_steps"] == wl.n_steps and g["dt"] == wl.rods[0][0].dt
    _say("c1 full: 2x512, 20000 steps at 10 per launch, shape (4,2)")
    b = R.RodBatch([s for s, _ in wl.rods])
    b.set_tuning(4, 2, 10)
    b.set_state_rods([st for _, st in wl.rods])
    tips = []
    for k in range(wl.n_steps // 1000):
        if k == wl.n_steps // 1000 - 1:
            b.step(990, 10)
            before = b.get_state_rods()
            b.step(10, 10)
        else:
            b.step(1000, 10)
        tips.append([x[-1].copy() for x, _, _, _ in b.get_state_rods()])
    b.sync()
    final = b.get_state_rods()
    b.close()
    for r, (spec, _) in enumerate(wl.rods):
        ref_tip = np.array(g["rods"][r]["tip"])
        got = np.array([t[r] for t in tips])
        err = np.linalg.norm(got - ref_tip, axis=1)
        _say("c1 rod %d: tip error every 1000 steps max %.2e final %.2e" % (r, err.max(), err[-1]))
        assert err.max() <= 1e-4 * 1.0
        sp = g["rods"][r]["sample_points"]
        ex = np.abs(final[r][0][sp] - np.array(g["rods"][r]["x"])).max()
        _say("c1 rod %d: sample points max|dx| %.2e" % (r, ex))
        assert ex <= 1e-4
        x = final[r][0].astype(np.float64)
        strain = np.abs(np.linalg.norm(np.diff(x, axis=0), axis=1) / spec.seg_len - 1).max()
        _say("c1 rod %d: max strain gpu %.2e oracle %.2e" % (r, strain, g["rods"][r]["max_strain"]))
        assert strain <= max(10 * g["rods"][r]["max_strain"], 1e-4)
    ref = oracle.rollout_many_threads(PM.fp32_rods(wl.rods), wl.n_steps - 10, n_threads=2)
    ref_b = [oracle.Rod(s).rollout(a, 10, t0=(wl.n_steps - 10) * s.dt)[0]
             for (s, _), a in zip(wl.rods, ref)]
    compare_window((before, final), (ref, ref_b), wl.rods, 10, "c1-full", PM.BARS["c1-full"])


_edge_rods = parity_cases.edge_rods


def test_edge_cases_mixed_batch(oracle):
    """One handle with ragged rods (N = 1, 2, 3, 65, 130, 200), both variants, clamped and
    free, driven clamps, external loads, intrinsic shape, non-uniform material."""
    rods = _edge_rods(oracle)
    ref = run_oracle_window(oracle, rods, 400, 37)
    for shape in ((4, 1), (2, 2), (1, 4)):
        _say("edge batch, 400 steps, shape %s" % (shape,))
        gpu = run_gpu_window(rods, 400, 37, 37, shape)
        compare_window(gpu, ref, rods, 37, "edge %s" % (shape,), PM.BARS["edge"])


def test_zero_steps_and_roundtrip():
    wl = W.config0()
    _say("state round trip")
    gpu = run_gpu(wl.rods, 0, 10)
    spec, st = wl.rods[0]
    x, v, q, w = gpu[0]
    assert np.array_equal(x, st.x.astype(np.float32)) and np.array_equal(q, st.q.astype(np.float32))


def test_launch_split_and_determinism_are_bitwise():
    wl = W.config1(n_steps=200)
    _say("c1 200 steps: 1x200 vs 20x10 vs 200x1 launches, repeated")
    a = run_gpu(wl.rods, 200, 200, (4, 2))
    b = run_gpu(wl.rods, 200, 10, (4, 2))
    c = run_gpu(wl.rods, 200, 1, (4, 2))
    d = run_gpu(wl.rods, 200, 10, (4, 2))
    for ra, rb, rc, rd in zip(a, b, c, d):
        for k in range(4):
            assert np.array_equal(ra[k], rb[k]) and np.array_equal(ra[k], rc[k])
            assert np.array_equal(rb[k], rd[k])


def _resume(rods, n1, n2, spl, shape):
    b = R.RodBatch([s for s, _ in rods])
    b.set_tuning(shape[0], shape[1], spl)
    b.set_state_rods([st for _, st in rods])
    b.step(n1, spl)
    x, v, q, w = b.get_state()
    t, steps = b.time()
    b.close()
    b = R.RodBatch([s for s, _ in rods])
    b.set_tuning(shape[0], shape[1], spl)
    b.set_state(x, v, q, w, t0=t)
    b.step(n2, spl)
    res = b.get_state_rods()
    b.close()
    return res


def test_checkpoint_resume():
    """get_state / set_state round trip mid-run.  The state the library hands out is FP32 (the
    low parts of the positions and quaternions stay inside the handle and restart at 0 after
    set_state), so a resumed run differs from a straight one by that one rounding: within
    1e-6 in x (m) and q."""
    for wl, label in ((W.config0(), "c0"), (W.config1(n_steps=300), "c1")):
        shape = (1, 1) if label == "c0" else (4, 2)
        _say("%s: 300 steps straight vs 120 + get/set + 180" % label)
        full = run_gpu(wl.rods, 300, 10, shape)
        res = _resume(wl.rods, 120, 180, 10, shape)
        for ra, rb in zip(full, res):
            dx = float(np.abs(ra[0] - rb[0]).max())
            dq = float(np.abs(ra[2] - rb[2]).max())
            _say("  %s resumed: max|dx| %.2e max|dq| %.2e" % (label, dx, dq))
            assert dx <= 1e-6 and dq <= 1e-6


def test_device_pointer_state_io():
    import torch
    wl = W.config0()
    spec, st = wl.rods[0]
    _say("device tensors in/out")
    b = R.RodBatch([spec])
    dev = [torch.tensor(a.astype(np.float32).ravel(), device="cuda") for a in (st.x, st.v, st.q, st.w)]
    b.set_state(*dev)
    b.step(50, 10)
    out = [torch.empty_like(t) for t in dev]
    b.get_state(out)
    torch.cuda.synchronize()
    host = b.get_state()
    b.close()
    for a, t in zip(host, out):
        assert np.array_equal(a, t.cpu().numpy())


def test_non_finite_state_is_reported():
    wl = W.config0()
    spec, st = wl.rods[0]
    _say("NaN in the state -> ROD_E_UNSTABLE")
    b = R.RodBatch([spec])
    x = st.x.astype(np.float32).ravel().copy()
    x[30] = np.nan
    b.set_state(x, st.v.astype(np.float32).ravel(), st.q.astype(np.float32).ravel(),
                st.w.astype(np.float32).ravel())
    b.step(10, 10)
    with pytest.raises(R.RodError) as e:
        b.sync()
    assert e.value.status == -4
    b.close()


def test_autotune_keeps_state_and_picks_a_shape():
    wl = W.config1(n_steps=100)
    _say("autotune on c1")
    b = R.RodBatch([s for s, _ in wl.rods])
    b.set_state_rods([st for _, st in wl.rods])
    before = b.get_state()
    t = b.autotune(probe_steps=100, steps_per_launch=10)
    after = b.get_state()
    assert b.time()[1] == 0
    b.close()
    _say("autotune chose %s" % t)
    assert 64 * t["waves"] * t["elems_per_lane"] >= 512 and t["us_per_step"] > 0
    for a, c in zip(before, after):
        assert np.array_equal(a, c)


def test_autotune_chooses_steps_per_launch(oracle):
    """steps_per_launch = 0: the autotuner also picks the steps per launch (state and step
    counter untouched); stepping with its choice matches the oracle."""
    wl = W.config0(n=64)
    spec, st = wl.rods[0]
    b = R.RodBatch([spec])
    b.set_state_rods([st])
    before = b.get_state()
    t = b.autotune(probe_steps=200, steps_per_launch=0)
    _say("autotune (steps per launch too) chose %s" % t)
    assert t["steps_per_launch"] in (1, 2, 5, 10, 20, 50, 100, 200)
    assert b.tuning["steps_per_launch"] == t["steps_per_launch"]
    after = b.get_state()
    assert b.time()[1] == 0
    for u, v in zip(before, after):
        assert np.array_equal(u, v)
    b.step(290)
    ga = b.get_state_rods()
    b.step(10)
    gb = b.get_state_rods()
    b.close()
    ref = run_oracle_window(oracle, wl.rods, 300, 10)
    compare_window((ga, gb), ref, wl.rods, 10, "autotuned c0", PM.BARS["c0"])


def test_batch_buckets_and_autotune_vs_oracle(oracle):
    """Uneven batch (per-rod dt from the stability rule, mixed variants) in several kernel-shape
    buckets, before and after autotuning, against the oracle rod by rod."""
    rods = parity_cases.batch48(oracle)
    b = R.RodBatch([s for s, _ in rods])
    bk = b.buckets()
    _say("batch of 48 rods (N 8..700) in buckets %s" % (bk,))
    assert len(bk) >= 3
    b.set_state_rods([st for _, st in rods])
    b.step(140, 70)
    ga = b.get_state_rods()
    b.step(10, 10)
    got = b.get_state_rods()
    b.set_state_rods([st for _, st in rods])
    t = b.autotune(probe_steps=20, steps_per_launch=70)
    _say("after autotune: %s, buckets %s" % (t, b.buckets()))
    b.step(140, 0)
    ga2 = b.get_state_rods()
    b.step(10, 0)
    got2 = b.get_state_rods()
    b.close()
    ref = run_oracle_window(oracle, rods, 150, 10)
    compare_window((ga, got), ref, rods, 10, "batch", PM.BARS["batch"])
    compare_window((ga2, got2), ref, rods, 10, "batch-tuned", PM.BARS["batch"])


def test_c3_full_size_sampled(oracle):
    """The full 4096-rod batch in the benchmark's launch configuration (autotuned shapes, 1000
    steps in one launch per bucket) against the oracle on sampled rods: every 256th rod, the
    costliest (longest inextensible) and the shortest.  The run's end: positions, tip, frames,
    window-mean velocities and unit quaternions.  The thin curved rods of the batch whip about
    (released from a curved shape towards a straight rest shape), and over 1000 steps that
    carries the FP32 noise of the force arithmetic into their Darboux vectors and body rates
    further than the FP32-storage floor: those two are held in 10-step windows restarted from
    the GPU's state at several steps, against bars from each window's floor."""
    wl = W.config3()
    rods = parity_cases.with_rule_dt(oracle, wl.rods)
    b = R.RodBatch([s for s, _ in rods])
    b.set_state_rods([st for _, st in rods])
    t = b.autotune(probe_steps=50, steps_per_launch=wl.n_steps)
    _say("c3 full: 4096 rods, %d steps in one launch per bucket; tuned %s, buckets %s"
         % (wl.n_steps, t, b.buckets()))
    pick = parity_cases.c3_pick(rods)
    sample = [rods[i] for i in pick]
    stops = (250, 500, 750, wl.n_steps - 10)
    at = {}
    for s in stops + (wl.n_steps,):   # each in one launch per bucket, as the benchmark runs
        b.set_state_rods([st for _, st in rods])
        b.step(s, s)
        got = b.get_state_rods()
        at[s] = [got[i] for i in pick]
        if s == wl.n_steps:
            for i, (x, v, q, w) in enumerate(got):   # every rod: finite, unit quaternions
                assert np.isfinite(x).all() and np.isfinite(v).all()
                assert np.abs(np.linalg.norm(q.astype(np.float64), axis=1) - 1).max() <= 1e-6, i
    b.close()
    ref = run_oracle_window(oracle, sample, wl.n_steps, 10)
    long_bars = {m: v for m, v in PM.BARS["c3"].items() if m not in ("u", "wbar")}
    compare_window((at[stops[-1]], at[wl.n_steps]), ref, sample, 10, "c3-sampled", long_bars)
    # restart windows: 10 steps from the GPU's states, on the GPU and on the oracle
    for s in stops:
        starts = [W.RodState(*[np.asarray(a, np.float64) for a in st]) for st in at[s]]
        gpu_b = []
        for r, ((spec, _), st) in enumerate(zip(sample, starts)):
            one = R.RodBatch([spec])
            one.set_state_rods([st], t0=s * spec.dt)
            one.step(10, 10)
            gpu_b.append(one.get_state_rods()[0])
            one.close()
        for r, ((spec, st0), g) in enumerate(zip(sample, gpu_b)):
            (S, pl, pert), = parity_cases.rod_restarts(oracle, spec, [starts[r]], [s])
            bars = PM.floor_bars(parity_cases.window_floor(spec, st0.x, S, pl, pert, 10, PM.errors))
            PM.check_window(([at[s][r]], [g]), ([S], [pl]), [(spec, st0)], 10,
                            "c3 rod %d from step %d" % (pick[r], s), bars, _say)


def test_first_multi_bucket_step_time_excludes_stream_setup():
    """The per-bucket streams are made on a handle's first multi-bucket step, outside the interval
    that rod_last_step_time() reports: the first step's time matches the next ones' (stream
    creation costs milliseconds, these steps tens of microseconds)."""
    wl = W.config3(n_rods=64, n_min=32, n_max=1500)
    rods = [(s.replace(dt=R.stable_dt(s)), st) for s, st in wl.rods]
    warm = R.RodBatch([s for s, _ in rods])   # first launches of these kernels: not timed here
    warm.set_state_rods([st for _, st in rods])
    warm.step(1, 1)
    warm.sync()
    warm.close()
    b = R.RodBatch([s for s, _ in rods])   # a new handle makes its own streams
    n_buckets = len(b.buckets())
    assert n_buckets >= 3
    b.set_state_rods([st for _, st in rods])
    times = []
    for _ in range(4):
        b.step(20, 20)
        b.sync()
        times.append(b.last_step_time()[0])
    b.close()
    _say("20-step times of a %d-bucket handle: %s ms" % (n_buckets, times))
    steady = float(np.median(times[1:]))
    assert times[0] < 3.0 * steady + 0.2, times
