"""Pins of the oracle's clamp force feedback (Sec. 2.2: the haptic thread reads a force-feedback
vector from the running simulation): the force the rod exerts on its clamped base point."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import workloads as W


def _masses(spec):
    r = O.Rod(spec)
    m = np.empty(spec.n + 1)
    for i in range(spec.n + 1):
        v = np.zeros((spec.n + 1, 3))
        v[i, 0] = 1.0
        m[i] = 2.0 * r.kinetic(v, np.zeros((spec.n, 3)))
    return m


@pytest.mark.parametrize("inext", [True, False])
@pytest.mark.parametrize("driven", [False, True])
def test_feedback_closes_the_momentum_balance(inext, driven):
    """Internal forces and constraint impulses act in opposite pairs, so over one step the
    momentum gained by points 1..n equals dt times their gravity, external loads and damping,
    minus dt times the force they pass to the clamped base point.  This fixes the feedback
    exactly, whatever the motion."""
    rng = np.random.default_rng(7)
    n = 12
    spec, st = W.straight_rod(n, inextensible=inext, dt=1e-4, damp=0.3)
    f_ext = rng.normal(0, 1e-3, (n + 1, 3))
    spec = spec.replace(f_ext=f_ext)
    if driven:
        spec = spec.replace(clamp_amp=(0.01, 0.0, 0.0), clamp_twist_amp=0.3, clamp_freq=3.0,
                            clamp_phase_x=0.4, clamp_phase_twist=1.1)
    st = st.copy()
    st.x = st.x + rng.normal(0, 1e-3, st.x.shape) * np.r_[0.0, np.ones(n)][:, None]
    st.v = rng.normal(0, 1e-2, st.v.shape)
    m = _masses(spec)
    g = np.asarray(spec.gravity)
    for t0 in (0.0, 0.37):
        new, fb = O.Rod(spec).rollout_fb(st, 1, t0=t0)
        dp = (m[1:, None] * (new.v[1:] - st.v[1:])).sum(axis=0)
        ext = (m[1:, None] * g[None, :] + f_ext[1:] - spec.damp_lin * m[1:, None] * st.v[1:]).sum(axis=0)
        expect = ext - dp / spec.dt
        scale = np.abs(dp / spec.dt).max() + np.abs(ext).max()
        assert np.abs(fb[0] - expect).max() <= 1e-9 * scale, (fb[0], expect)


def test_hanging_rod_pulls_with_its_weight():
    """A straight inextensible rod hanging from its clamp, at rest: the feedback is the weight of
    everything below the clamped point."""
    n = 8
    spec, st = W.straight_rod(n, inextensible=True, dt=1e-4, n_iter=400, damp=1.0,
                              q0=(0.0, 1.0, 0.0, 0.0))      # third axis pointing down (-z)
    assert np.allclose(st.x[-1], [0.0, 0.0, -1.0])
    m = _masses(spec)
    _, fb = O.Rod(spec).rollout_fb(st, 50)
    weight = (m[1:].sum()) * np.asarray(spec.gravity)
    assert np.abs(fb[-1] - weight).max() <= 1e-6 * np.abs(weight).max()
