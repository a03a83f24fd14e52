"""GPU parity of the chunked long-rod kernel (one workgroup per chunk of about 500 elements,
halo exchange through global memory every few steps) against the FP64 oracle and against the
single-workgroup kernel on the same rod.  Runs are compared as whole states (parity_metrics):
positions, tip within 1e-4 x rod length, frames, Darboux vectors and window-mean velocities.
"""
import os
import sys

import numpy as np
import pytest

from paper_2509_04277_amd import rod as R
from paper_2509_04277_amd import workloads as W
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
    torch.cuda.init()
    yield


def _run(rods, n_steps, spl, chunk_above=None, chunk=0, splits=None, shape=None, window=0):
    """GPU run; with window = k > 0 also the state k steps before the end (returned as the
    pair (before, end) in place of the end state)."""
    b = R.RodBatch([s for s, _ in rods])
    if shape is not None:
        b.set_tuning(shape[0], shape[1], spl)
    if chunk_above is not None:
        b.set_chunking(chunk_above, chunk)
    b.set_state_rods([st for _, st in rods])
    if window:
        b.step(n_steps - window, spl)
        before = b.get_state_rods()
        b.step(window, spl)
    else:
        for k in (splits or [n_steps]):
            b.step(k, spl)
    b.sync()
    out = b.get_state_rods()
    info = b.buckets()
    b.close()
    return ((before, out) if window else out), info


def _vs_oracle(oracle, rods, gpu, n_steps, k, label, tol=None):
    """Whole-state comparison (parity_metrics) of a windowed GPU run with the oracle."""
    errs = []
    for r, (s, st) in enumerate(rods):
        a = oracle.Rod(s).rollout(PM.fp32_input(st), n_steps - k)[0]
        c = oracle.Rod(s).rollout(a, k, t0=(n_steps - k) * s.dt)[0]
        assert all(np.isfinite(v).all() for v in gpu[1][r])
        e = PM.errors(s, st.x, gpu[0][r], gpu[1][r], (a.x, a.v, a.q, a.w), (c.x, c.v, c.q, c.w), k)
        _say("%s N=%d %s: %s" % (label, s.n, "inext" if s.inextensible else "ext", PM.fmt(e)))
        errs.append(e)
    bad = PM.violations(PM.worst(errs), tol)
    assert not bad, "%s: above the bars: %s" % (label, bad)


@pytest.mark.parametrize("case", ["c2-500-inext", "c2-500-ext", "c1-2x512-driven"])
def test_chunked_is_bitwise_single_workgroup(case):
    """Chunked and single-workgroup kernels of the same shape (4 waves x 2 elements per lane)
    on the same rods: windows start at even elements, so every owned element is computed by
    the same instructions from the same operands, and the halo (2 n_iter + 4 elements per
    side) covers one step's dependency radius.  Any halo shortfall breaks bitwise equality."""
    if case == "c1-2x512-driven":
        rods, chunk = W.config1().rods, 128
    else:
        rods, chunk = W.config2(500, case.endswith("-inext")).rods, 64
    n_steps = 300
    one, info1 = _run(rods, n_steps, 10, shape=(4, 2))
    many, info2 = _run(rods, n_steps, 10, chunk_above=1, chunk=chunk)
    _say("%s: %d steps; buckets single %s, chunked %s" % (case, n_steps, info1, info2))
    assert info1 == [(4, 2, len(rods), 0.0)] and info2 == [(4, 2, len(rods), 0.0)]
    for r, (a, b) in enumerate(zip(one, many)):
        d = [float(np.abs(u - v).max()) for u, v in zip(a, b)]
        _say("  rod %d max diffs x %.2e v %.2e q %.2e w %.2e" % (r, *d))
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


@pytest.mark.parametrize("inext,chunk", [(True, 0), (False, 0), (True, 60), (False, 60)])
def test_chunked_matches_wider_single_workgroup(oracle, inext, chunk):
    """A 2000-element rod in 5 chunks (or 34 of about 60 elements, most neighbours on other
    XCDs) against the same rod in one 8-wave x 4-element workgroup: multiply-adds are fused
    only within a source expression, so the grouping of elements into lanes does not change
    any element's arithmetic, and the halo exchange must deliver every neighbour value."""
    wl = W.config2(2000, inext)
    L = float(np.sum(wl.rods[0][0].seg_len))
    n_steps = 300
    one, info1 = _run(wl.rods, n_steps, 10)
    (many_a, many), info2 = _run(wl.rods, n_steps, 10, chunk_above=1024, chunk=chunk, window=10)
    _say("1x2000 %s, %d steps, chunk %d; buckets single %s, chunked %s"
         % ("inext" if inext else "ext", n_steps, chunk, info1, info2))
    assert info2 == [(4, 2, 1, 0.0)]
    (x1, v1, q1, w1), (x2, v2, q2, w2) = one[0], many[0]
    dx, dq = np.abs(x1 - x2).max(), np.abs(q1 - q2).max()
    _say("  max diffs: x %.2e (L %.1f) q %.2e v %.2e w %.2e" % (
        dx, L, dq, np.abs(v1 - v2).max(), np.abs(w1 - w2).max()))
    for u, v in zip(one[0], many[0]):
        assert np.array_equal(u, v)
    _vs_oracle(oracle, wl.rods, (many_a, many), n_steps, 10, "chunked-2000", PM.BARS["c2"])


def test_every_kernel_shape_is_bitwise():
    """The two c1 rods (512 elements, driven clamp) in every built shape that holds them and
    in 4 chunks: identical states after 300 steps."""
    rods = W.config1().rods
    ref, _ = _run(rods, 300, 10, shape=(4, 2))
    for shape in [(1, 8), (2, 4), (8, 1), (4, 4), (8, 2), (4, 8), (8, 4), (16, 1)]:
        got, _ = _run(rods, 300, 10, shape=shape)
        same = all(np.array_equal(u, v) for a, b in zip(ref, got) for u, v in zip(a, b))
        _say("shape %s bitwise equal to (4, 2): %s" % (shape, same))
        assert same
    got, _ = _run(rods, 300, 10, chunk_above=1, chunk=128)
    assert all(np.array_equal(u, v) for a, b in zip(ref, got) for u, v in zip(a, b))


@pytest.mark.parametrize("inext", [True, False])
def test_c2_4096_full_run(oracle, inext):
    wl = W.config2(4096, inext)
    _say("c2 full: 1x4096 %s, %d steps at %d per launch"
         % ("inext" if inext else "ext", wl.n_steps, wl.steps_per_launch))
    gpu, info = _run(wl.rods, wl.n_steps, wl.steps_per_launch, window=10)
    assert info == [(4, 2, 1, 0.0)]
    _vs_oracle(oracle, wl.rods, gpu, wl.n_steps, 10, "c2-4096", PM.BARS["c2"])


@pytest.mark.parametrize("n", [16384, 65536])
@pytest.mark.parametrize("inext", [True, False])
def test_c2_full_run_against_stored_oracle(n, inext):
    """The long-rod workload at 16384 and 65536 elements over its 5000 steps (chunked, 100 steps
    per launch) against the stored FP64 oracle (tests/golden/make_c2_golden.py): 32 pieces of
    8 consecutive elements along the rod, the last at the tip, compared as whole states."""
    g = np.load(os.path.join(HERE, "golden", "c2_oracle_%d_%s.npz" % (n, "inext" if inext else "ext")))
    wl = W.config2(n, inext)
    spec, st = wl.rods[0]
    k = int(g["window"])
    assert int(g["n_steps"]) == wl.n_steps and float(g["dt"]) == spec.dt and int(g["n"]) == n
    _say("c2 full: 1x%d %s, %d steps at 100 per launch" % (n, "inext" if inext else "ext", wl.n_steps))
    (before, end), _ = _run(wl.rods, wl.n_steps, 100, window=k)
    L = float(np.sum(spec.seg_len))
    errs = []
    for i, p0 in enumerate(g["starts"]):
        pt, fr = slice(p0, p0 + 9), slice(p0, p0 + 8)
        got = [(x[pt], v[pt], q[fr], w[fr]) for x, v, q, w in (before[0], end[0])]
        ref = [(g["xa"][i], None, g["qa"][i], None), (g["xb"][i], None, g["qb"][i], None)]
        errs.append(PM.errors(spec, st.x[pt], got[0], got[1], ref[0], ref[1], k,
                              seg_len=spec.seg_len[fr], disp=float(g["disp"]), length=L))
    tip = float(np.linalg.norm(end[0][0][-1] - g["xb"][-1][-1])) / L
    w = PM.worst(errs)
    w["tip"] = tip
    _say("c2-%d %s (32 pieces): %s" % (n, "inext" if inext else "ext", PM.fmt(w)))
    bad = PM.violations(w, PM.BARS["c2"])
    assert not bad, bad


def test_longest_accepted_rod_short_run(oracle):
    """The longest rod a handle accepts (2^17 elements, 283 chunks resident together), 50 steps
    at 25 per launch, every point against the oracle."""
    wl = W.config2(1 << 17, True)
    _say("longest rod: 1x131072 inext, 50 steps at 25 per launch")
    gpu, info = _run(wl.rods, 50, 25, window=25)
    assert info == [(4, 2, 1, 0.0)]
    _vs_oracle(oracle, wl.rods, gpu, 50, 25, "c2-131072", PM.BARS["c2"])


def test_autotune_chunks_a_lone_long_rod(oracle):
    """rod_autotune with steps_per_launch = 0 times a lone 2048-element rod in one workgroup and
    chunked, keeps the faster (chunked: about 5 against 8.5 us per step), leaves state and step
    counter as they were, and the rod then steps as the oracle does."""
    wl = W.config2(2048, True)
    spec, st = wl.rods[0]
    b = R.RodBatch([spec])
    b.set_state_rods([st])
    before = b.get_state()
    t = b.autotune(probe_steps=100, steps_per_launch=0)
    info = b.buckets()
    _say("autotune on 1x2048 inext chose %s, buckets %s" % (t, info))
    assert info == [(4, 2, 1, 0.0)]   # the chunked long-rod bucket
    assert b.time()[1] == 0
    for u, v in zip(before, b.get_state()):
        assert np.array_equal(u, v)
    b.step(290)
    gpu_a = b.get_state_rods()
    b.step(10)
    b.sync()
    gpu = b.get_state_rods()
    b.close()
    _vs_oracle(oracle, wl.rods, (gpu_a, gpu), 300, 10, "autotuned-2048", PM.BARS["c2"])


def test_launch_split_and_restart_are_bitwise():
    """Chunk flags carry absolute step numbers across launches; rod_set_state restarts them."""
    wl = W.config2(4096, True)
    _say("c2 1x4096 inext: 100 steps as 1x100 (k=100), 100x1 (k=1), 10x10 (k=10), restarted")
    b = R.RodBatch([s for s, _ in wl.rods])
    res = []
    for spl in (100, 1, 10):
        b.set_state_rods([st for _, st in wl.rods])
        b.step(100, spl)
        b.sync()
        res.append(b.get_state_rods()[0])
        _say("  k=%d done" % spl)
    b.close()
    for other in res[1:]:
        for a, c in zip(res[0], other):
            assert np.array_equal(a, c)


def test_chunked_handles_on_two_streams_are_bitwise_alone():
    """Two handles with chunked rods on two streams, stepped in interleaved calls: the library
    orders their chunked runs (each grid has the device to itself), and each handle ends
    bitwise where it ends alone."""
    import torch
    rods = [W.config2(16384, True).rods[0], W.config2(9000, False).rods[0]]
    alone = [_run([r], 300, 10)[0][0] for r in rods]
    streams = [torch.cuda.Stream() for _ in rods]
    hs = []
    for r, s in zip(rods, streams):
        h = R.RodBatch([r[0]], stream=s.cuda_stream)
        h.set_state_rods([r[1]])
        hs.append(h)
    _say("two handles (1x16384 inext, 1x9000 ext) on two streams, 3 x 100 steps each, interleaved")
    for _ in range(3):
        for h in hs:
            h.step(100, 10)
    got = []
    for h in hs:
        h.sync()
        got.append(h.get_state_rods()[0])
        h.close()
    for a, b in zip(got, alone):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_mixed_handle_long_and_short(oracle):
    """One handle holding resident rods and a chunked rod: one rod_step advances all."""
    rods = W.config0().rods + W.config2(3000, True).rods + W.config2(700, False).rods
    _say("mixed handle: N=64 ext, N=3000 inext (chunked), N=700 ext; 500 steps")
    gpu, info = _run(rods, 500, 10, window=10)
    _say("buckets %s" % info)
    assert info[-1][:3] == (4, 2, 1)
    _vs_oracle(oracle, rods, gpu, 500, 10, "mixed", PM.BARS["c2"])


def test_set_chunking_arguments():
    wl = W.config2(1000, True)
    b = R.RodBatch([s for s, _ in wl.rods])
    for bad in (0, -1, 2049):
        with pytest.raises(R.RodError):
            b.set_chunking(bad)
    with pytest.raises(R.RodError):
        b.set_chunking(10, -1)
    b.set_chunking(2048)
    assert b.buckets()[-1][2] == 1 and len(b.buckets()) == 1
    b.set_chunking(999)
    assert b.buckets() == [(4, 2, 1, 0.0)]
    b.set_chunking(999, 1)   # clamped up to the smallest chunk, 2 H + 2 = 50
    b.set_state_rods([st for _, st in wl.rods])
    b.step(10, 10)
    b.sync()
    b.close()
