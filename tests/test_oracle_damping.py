"""Pins of the oracle's internal friction (Sec. 2.1: the CoRdE model's dissipation terms that
damp relative motion, translational and angular; read as Kelvin-Voigt, the Rayleigh function
being the elastic energy's quadratic form at the strain rates), against what the definition
and mechanics fix."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2509_04277_amd import workloads as W


def _random_rod(inext, td, seed=3, n=8):
    rng = np.random.default_rng(seed)
    x, q = W.curved_rod(n, 0.05, rng, 0.3, twist_sigma=0.2)
    spec, _ = W.straight_rod(n, L=0.4, inextensible=inext, dt=1e-5)
    spec = spec.replace(damp_int=td, young=rng.uniform(1e6, 3e6, n), radius=rng.uniform(5e-3, 1e-2, n),
                        seg_len=np.linalg.norm(np.diff(x, axis=0), axis=1))
    v = rng.normal(size=(n + 1, 3))
    w = rng.normal(size=(n, 3))
    return spec, x, q, v, w


@pytest.mark.parametrize("inext", [False, True])
def test_forces_are_minus_the_velocity_gradient(inext):
    """F = -dD/dv and tau = -dD/domega by central differences of the dissipation function."""
    spec, x, q, v, w = _random_rod(inext, 2e-3)
    rod = O.Rod(spec)
    F, tau = rod.damping_forces(x, q, v, w)
    h = 1e-6
    for i in range(spec.n + 1):
        for c in range(3):
            vp, vm = v.copy(), v.copy()
            vp[i, c] += h
            vm[i, c] -= h
            g = (rod.dissipation(x, q, vp, w) - rod.dissipation(x, q, vm, w)) / (2 * h)
            assert abs(F[i, c] + g) <= 1e-6 * (1 + abs(g))
    for j in range(spec.n):
        for c in range(3):
            wp, wm = w.copy(), w.copy()
            wp[j, c] += h
            wm[j, c] -= h
            g = (rod.dissipation(x, q, v, wp) - rod.dissipation(x, q, v, wm)) / (2 * h)
            assert abs(tau[j, c] + g) <= 1e-6 * (1 + abs(g))
    # D is quadratic in the velocities: the damping power is -2 D
    P = np.sum(F * v) + np.sum(tau * w)
    assert abs(P + 2 * rod.dissipation(x, q, v, w)) <= 1e-10 * abs(P)
    if inext:   # no stretch term: point forces vanish
        assert not F.any()


def test_rigid_motion_is_not_damped():
    """A rigid motion of a curved, twisted rod (v = V + Omega x x, body omega = R^T Omega) changes
    no strain: no dissipation, no forces."""
    spec, x, q, _, _ = _random_rod(False, 5e-3)
    rod = O.Rod(spec)
    V, Om = np.array([0.3, -0.2, 0.1]), np.array([1.5, -0.7, 2.0])
    v = V + np.cross(Om, x)
    w = np.array([O.rotmat(qj).T @ Om for qj in q])
    F, tau = rod.damping_forces(x, q, v, w)
    assert rod.dissipation(x, q, v, w) <= 1e-24
    assert np.abs(F).max() <= 1e-12 and np.abs(tau).max() <= 1e-14
    # and a stretching / bending motion is damped
    _, _, _, v2, w2 = _random_rod(False, 5e-3)
    assert rod.dissipation(x, q, v2, w2) > 0


def test_axial_vibration_decays_as_kelvin_voigt():
    """One free extensible element stretched and released: a mass-spring-damper with spring
    K_s / l, dashpot tau_d K_s / l and reduced mass m / 4, whose amplitude decays as
    exp(-tau_d omega^2 t / 2)."""
    L, r, E, rho = 0.1, 5e-3, 1e6, 1000.0
    spec, st = W.straight_rod(1, L=L, radius=r, young=E, inextensible=False, gravity=(0, 0, 0),
                              clamp=False, dt=1e-6)
    A = np.pi * r * r
    m = rho * A * L
    w0 = np.sqrt((E * A / L) / (m / 4))
    td = 0.02 / w0                                   # damping ratio 1 %
    spec = spec.replace(damp_int=td, dt=2 * np.pi / w0 / 400)
    st = st.copy()
    st.x = st.x * np.array([1.0, 1.0, 1.0])
    st.x[1] = st.x[0] + (st.x[1] - st.x[0]) * 1.01   # 1 % stretch
    rod = O.Rod(spec)
    n_per = 400
    amps = []
    s = st
    for period in range(6):
        s, _ = rod.rollout(s, n_per)
        amps.append(np.linalg.norm(s.x[1] - s.x[0]) / L - 1.0)
    ratio = amps[-1] / amps[0]
    T = 2 * np.pi / w0
    want = np.exp(-td * w0 ** 2 * 5 * T / 2)
    assert abs(ratio / want - 1) <= 0.02, (ratio, want)
    # without internal friction the amplitude is kept
    s0, _ = O.Rod(spec.replace(damp_int=0.0)).rollout(st, 5 * n_per)
    assert abs((np.linalg.norm(s0.x[1] - s0.x[0]) / L - 1.0) / 0.01 - 1) <= 0.02


def test_dt_rule_includes_the_dampers():
    """With a strong damper the rule's dt shrinks as 2 / (tau_d omega^2); the run stays bounded
    at the rule and blows up at 4x."""
    spec, st = W.straight_rod(8, L=0.4, inextensible=False, dt=1e-5, gravity=(0, 0, -9.81))
    d0 = O.Rod(spec).dt_rule()
    strong = spec.replace(damp_int=50 * d0)
    d1 = O.Rod(strong).dt_rule()
    assert d1 < 0.1 * d0
    st = st.copy()
    st.v = np.random.default_rng(2).normal(0, 0.1, st.v.shape)
    assert O.Rod(strong.replace(dt=d1)).stable(st, 2000)
    assert not O.Rod(strong.replace(dt=4 * d1)).stable(st, 2000)


def test_twist_vibration_decays_as_kelvin_voigt():
    """Two free frames twisted against each other about the rod axis: a torsion spring K_3 / lbar,
    dashpot tau_d K_3 / lbar and reduced inertia I_3 / 2, decaying as exp(-tau_d omega^2 t / 2)."""
    L, r, E, rho = 0.1, 5e-3, 1e6, 1000.0
    spec, st = W.straight_rod(2, L=L, radius=r, young=E, inextensible=False, gravity=(0, 0, 0),
                              clamp=False, dt=1e-6)
    l = L / 2
    m = rho * np.pi * r * r * l
    I3 = m * r * r / 2
    G = E / (2 * (1 + 0.5))
    K3 = G * np.pi * r ** 4 / 2
    w0 = np.sqrt((K3 / l) / (I3 / 2))
    td = 0.02 / w0
    spec = spec.replace(damp_int=td, dt=2 * np.pi / w0 / 400)
    st = st.copy()
    th = 0.02
    rot = np.array([np.cos(th / 2), 0.0, 0.0, np.sin(th / 2)])   # about body axis 3
    st.q = st.q.copy()
    st.q[1] = W._qprod(st.q[1], rot)
    rod = O.Rod(spec)

    def twist(s):
        return 2 * np.arctan2(rod.darboux(s.q, 0)[2] * l / 2, 1.0)

    a0 = twist(st)
    s, _ = rod.rollout(st, 5 * 400)
    # amplitude after 5 periods (the twist is back at an extreme)
    ratio = twist(s) / a0
    want = np.exp(-td * w0 ** 2 * 5 * (2 * np.pi / w0) / 2)
    assert abs(ratio / want - 1) <= 0.02, (ratio, want)
