"""Pins of the oracle's contact (Sec. 2.2 "Collisions and self-collisions": sphere-sphere
contact between mass points of two rods or of one rod; Sec. 2.1: contact constraints with
Coulomb friction solved as impulses), checked against what the definition fixes."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import workloads as W


def _cross(gap=0.9, vb=(0.0, 0.0, 0.0), n=2, l=0.05, r=0.01, n_iter=10):
    """Two free 2-element rods crossing at their middle points (A along x, B along y above
    it); the middle spheres overlap (distance gap * 2r), no other pair does."""
    a, sa = W.straight_rod(n, L=n * l, radius=r, inextensible=True, dt=1e-4, gravity=(0, 0, 0),
                           clamp=False, n_iter=n_iter)
    b, sb = W.straight_rod(n, L=n * l, radius=r, inextensible=True, dt=1e-4, gravity=(0, 0, 0),
                           clamp=False, q0=(np.cos(np.pi / 4), -np.sin(np.pi / 4), 0.0, 0.0),
                           n_iter=n_iter)
    sa, sb = sa.copy(), sb.copy()
    sa.x = sa.x - sa.x[1]                      # A's middle point at the origin
    sb.x = sb.x - sb.x[1] + np.array([0.0, 0.0, gap * 2 * r])
    sb.v = np.tile(np.asarray(vb, dtype=np.float64), (n + 1, 1))
    return [a, b], [sa, sb]


def _momentum(spec, st):
    r = O.Rod(spec)
    m = np.empty(spec.n + 1)
    for i in range(spec.n + 1):
        v = np.zeros((spec.n + 1, 3))
        v[i, 0] = 1.0
        m[i] = 2.0 * r.kinetic(v, np.zeros((spec.n, 3)))
    return (m[:, None] * st.v).sum(axis=0)


def test_single_contact_resolves_penetration_and_keeps_momentum():
    specs, states = _cross(gap=0.9)
    (A, B), most = O.rollout_group(specs, states, 1, mu=0.0)
    assert most == 1
    # the contact impulse is the last constraint of the last iteration: the points end exactly
    # at the target distance along the start-of-step normal
    d = A.x[1] - B.x[1]
    assert abs(-d[2] - 2 * 0.01) <= 1e-12
    p0 = _momentum(specs[0], states[0]) + _momentum(specs[1], states[1])
    p1 = _momentum(specs[0], A) + _momentum(specs[1], B)
    moved = np.abs(_momentum(specs[1], B) - _momentum(specs[1], states[1])).max()
    assert moved > 1e-6
    assert np.abs(p1 - p0).max() <= 1e-12 * moved


def test_separated_spheres_do_not_interact():
    specs, states = _cross(gap=1.01)
    (A, B), most = O.rollout_group(specs, states, 3, mu=0.5)
    (A0, B0), _ = O.rollout_group(specs, states, 3)
    assert most == 0
    for u, v in ((A.x, A0.x), (A.v, A0.v), (B.x, B0.x), (B.q, B0.q)):
        assert np.array_equal(u, v)


@pytest.mark.parametrize("mu", [0.0, 1e6])
def test_coulomb_friction(mu):
    """B slides along x over A.  Without friction the contact leaves the tangential motion
    alone; with unbounded friction the contact points end with no relative tangential
    velocity (sticking: with one constraint iteration the contact is the last impulse and is
    active), and momentum is kept either way."""
    specs, states = _cross(gap=0.9, vb=(0.1, 0.0, 0.0), n_iter=1)
    (A, B), most = O.rollout_group(specs, states, 1, mu=mu)
    assert most == 1
    vr = B.v[1] - A.v[1]
    vt = vr - vr[2] * np.array([0.0, 0.0, 1.0])
    if mu == 0.0:
        # the contact adds no tangential impulse; A's own distance constraints (its middle point
        # is pushed down at ~10 m/s) leave only a rounding-level x velocity on it
        assert abs(vt[0] - 0.1) <= 1e-8 and abs(A.v[1][0]) <= 1e-8
    else:
        assert np.abs(vt).max() <= 1e-12
        assert A.v[1][0] > 1e-3                 # A was dragged along
    p0 = _momentum(specs[0], states[0]) + _momentum(specs[1], states[1])
    p1 = _momentum(specs[0], A) + _momentum(specs[1], B)
    moved = np.abs(_momentum(specs[1], B) - _momentum(specs[1], states[1])).max()
    assert np.abs(p1 - p0).max() <= 1e-13 * moved


def test_straight_rod_has_no_self_contact():
    """Neighbouring points overlap at rest (radius 1 cm, element 1/64 m) but are excluded."""
    spec, st = W.straight_rod(64, radius=0.01, inextensible=True, dt=1e-5)
    assert O.self_skip(spec) == 2
    _, most = O.rollout_group([spec], [st], 5, mu=0.3)
    assert most == 0
    _, most = O.rollout_group([spec.replace(radius=np.full(64, 0.02))], [st], 1, mu=0.3)
    assert most == 0


def coiled(n=48, turns=2, L=1.0, r=0.01, rise=0.5):
    """Two flat turns of a circle with a slight helical rise: the second turn lies on the first,
    its points `rise` x 2r above; the rest shape (intrinsic curvature) is this shape."""
    R = L / (2 * np.pi * turns)
    s = np.linspace(0.0, L, n + 1)
    x = np.stack([R * np.sin(s / R), R * (1 - np.cos(s / R)), rise * 2 * r * s / (L / turns)], 1)
    q = W.frames_from_polyline(x)
    spec, st = W.straight_rod(n, L=L, radius=r, inextensible=True, dt=1e-5, gravity=(0, 0, 0),
                              damp=5.0)
    rod = O.Rod(spec)
    u_hat = np.array([rod.darboux(q, j) for j in range(n - 1)])
    lens = np.linalg.norm(x[1:] - x[:-1], axis=1)
    spec = spec.replace(u_hat=u_hat, seg_len=lens, clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    spec = spec.replace(dt=O.Rod(spec).dt_rule())
    st = st.copy()
    st.x, st.q = x, q
    return spec, st


def _closest(x, skip):
    n = x.shape[0] - 1
    return min(np.linalg.norm(x[i] - x[j]) for i in range(1, n + 1)
               for j in range(i + skip + 1, n + 1))


def test_coiled_rod_self_contact_keeps_turns_apart():
    """The rest shape puts the second turn on the first (25 % of the contact distance above
    it): without contact the rod stays there; with contact the turns are pushed apart to the
    sum of the radii."""
    spec, st = coiled()
    skip = O.self_skip(spec)
    free, most0 = O.rollout_group([spec], [st], 200)
    touched, most = O.rollout_group([spec], [st], 200, mu=0.2)
    assert most0 == 0 and most >= 1
    assert _closest(free[0].x, skip) < 0.5 * 2 * 0.01
    assert _closest(touched[0].x, skip) >= 0.98 * 2 * 0.01
