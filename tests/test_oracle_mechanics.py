"""Pins of the oracle's mechanics against what the model and textbook mechanics fix.

Energies are those of Sec. 2.1 (eqs. (2), (3), (8)); forces and torques must be their exact
negative gradients; the discrete rod must reproduce the static closed forms of linear
elasticity (axial extension P L / (E A), torsion T L / (G J), Euler-Bernoulli cantilever sag
w L^4 / (8 E I) and tip deflection P L^3 / (3 E I)) and the first cantilever frequency
(1.875^2 / 2 pi) sqrt(E I / (rho A L^4)); a straight unloaded rod must stay at rest; internal
forces must be invariant under rigid motions; quaternions stay unit; inextensibility impulses
converge to exact lengths.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation as Rot

from paper_2509_04277_amd import workloads as W


def _from_sp(r):
    x, y, z, w = r.as_quat()
    return np.array([w, x, y, z])


def _noisy_rod(n=7, inext=False, seed=20, uhat=True):
    """Small curved rod with non-uniform material, gravity, intrinsic shape and noisy frames."""
    rng = np.random.default_rng(seed)
    x, q = W.curved_rod(n, 0.05, rng, sigma=0.3, twist_sigma=0.2)
    x[1:] += rng.normal(0, 2e-3, size=(n, 3))
    q = q + rng.normal(0, 0.05, size=q.shape)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    spec = W.RodSpec(
        n=n, inextensible=inext, n_iter=5, clamp=True, dt=1e-5, gravity=(0.3, -1.0, -9.81),
        damp_lin=0.0, damp_ang=0.0, poisson=0.3, density=1200.0,
        seg_len=rng.uniform(0.04, 0.06, n), radius=rng.uniform(0.005, 0.01, n),
        young=rng.uniform(1e5, 1e6, n), kp_scale=0.7, bend_scale=1.3, twist_scale=0.8,
        u_hat=rng.normal(0, 2.0, size=(n - 1, 3)) if uhat else None,
        f_ext=rng.normal(0, 0.1, size=(n + 1, 3)),
        clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]))
    v = rng.normal(0, 0.1, size=(n + 1, 3))
    w = rng.normal(0, 1.0, size=(n, 3))
    return spec, W.RodState(x, v, q, w)


@pytest.mark.parametrize("inext", [False, True])
def test_forces_are_negative_energy_gradient(oracle, inext):
    spec, st = _noisy_rod(inext=inext)
    rod = oracle.Rod(spec)
    F, tau = rod.forces(st.x, st.q)
    h = 1e-7
    Ffd = np.zeros_like(F)
    for i in range(spec.n + 1):
        for c in range(3):
            xp, xm = st.x.copy(), st.x.copy()
            xp[i, c] += h
            xm[i, c] -= h
            Ffd[i, c] = -(rod.energy(xp, st.q) - rod.energy(xm, st.q)) / (2 * h)
    scale = np.abs(F).max()
    assert np.abs(F - Ffd).max() <= 1e-6 * scale
    # torque about body axis a: -dV/d eps of q (x) exp(eps e_a / 2)
    eps = 1e-6
    tfd = np.zeros_like(tau)
    for j in range(spec.n):
        for a in range(3):
            qp, qm = st.q.copy(), st.q.copy()
            rv = np.zeros(3)
            rv[a] = eps
            qp[j] = oracle.qmul(st.q[j], _from_sp(Rot.from_rotvec(rv)))
            qm[j] = oracle.qmul(st.q[j], _from_sp(Rot.from_rotvec(-rv)))
            tfd[j, a] = -(rod.energy(st.x, qp) - rod.energy(st.x, qm)) / (2 * eps)
    tscale = np.abs(tau).max()
    assert np.abs(tau - tfd).max() <= 1e-6 * tscale


def test_rigid_motion_invariance(oracle):
    spec, st = _noisy_rod(seed=21)
    spec = spec.replace(gravity=(0.0, 0.0, 0.0), f_ext=None)
    rod = oracle.Rod(spec)
    V0 = rod.energy(st.x, st.q)
    F0, t0 = rod.forces(st.x, st.q)
    rng = np.random.default_rng(22)
    for _ in range(5):
        R = Rot.from_quat(rng.normal(size=4))
        c = rng.normal(size=3)
        x2 = st.x @ R.as_matrix().T + c
        rq = _from_sp(R)
        q2 = np.stack([oracle.qmul(rq, qj) for qj in st.q])
        assert abs(rod.energy(x2, q2) - V0) <= 1e-12 * abs(V0)
        F2, t2 = rod.forces(x2, q2)
        assert np.abs(F2 - F0 @ R.as_matrix().T).max() <= 1e-11 * np.abs(F0).max()
        assert np.abs(t2 - t0).max() <= 1e-11 * np.abs(t0).max()
        # internal forces sum to zero (Newton's third law)
        assert np.abs(F2.sum(axis=0)).max() <= 1e-12 * np.abs(F0).max()


@pytest.mark.parametrize("inext", [False, True])
def test_rest_state_stays_at_rest(oracle, inext):
    q0 = _from_sp(Rot.from_rotvec([0.3, -1.1, 0.4]))
    spec, st = W.straight_rod(16, L=0.8, inextensible=inext, gravity=(0, 0, 0), damp=0.1,
                              q0=q0, dt=1e-4)
    rod = oracle.Rod(spec)
    F, tau = rod.forces(st.x, st.q)
    assert np.abs(F).max() < 1e-12 and np.abs(tau).max() < 1e-12
    out, _ = rod.rollout(st, 10000)
    assert np.abs(out.x - st.x).max() < 1e-13
    assert np.abs(out.q - st.q).max() < 1e-13
    assert np.abs(out.v).max() < 1e-12 and np.abs(out.w).max() < 1e-10


def test_unit_quaternions_after_steps(oracle):
    wl = W.config0(dt=1e-4)
    spec, st = wl.rods[0]
    out, _ = oracle.Rod(spec).rollout(st, 500)
    assert np.abs(np.linalg.norm(out.q, axis=1) - 1.0).max() <= 1e-14


def test_constraint_iterations_converge_to_exact_lengths(oracle):
    """With all elastic and external forces off, the impulses alone restore rest lengths."""
    rng = np.random.default_rng(23)
    n = 8   # red-black sweeps on a chain contract like cos^2(pi / (2n + 1)) per iteration
    spec, st = W.straight_rod(n, L=1.0, inextensible=True, gravity=(0, 0, 0), dt=1e-3,
                              n_iter=2000, clamp=True)
    spec = spec.replace(kp_scale=0.0, bend_scale=0.0, twist_scale=0.0)
    st.v = rng.normal(0, 0.5, size=st.v.shape)
    rod = oracle.Rod(spec)
    out, _ = rod.rollout(st, 1)
    assert rod.max_strain(out.x) < 1e-12
    # one iteration: the last (odd) half-sweep leaves odd segments exactly at rest length
    out1, _ = oracle.Rod(spec.replace(n_iter=1)).rollout(st, 1)
    lens = np.linalg.norm(np.diff(out1.x, axis=0), axis=1)
    assert np.abs(lens[1::2] / spec.seg_len[1::2] - 1).max() < 1e-12
    assert np.abs(lens[0::2] / spec.seg_len[0::2] - 1).max() > 1e-6


def _relax(oracle, spec, st, n_steps, chunk=5000, tol=1e-10):
    rod = oracle.Rod(spec)
    s = st
    for k in range(0, n_steps, chunk):
        s2, _ = rod.rollout(s, chunk)
        moved = max(np.abs(s2.x - s.x).max(), np.abs(s2.q - s.q).max())
        s = s2
        if moved < tol:
            break
    return s


def test_axial_extension_closed_form(oracle):
    """Static tip load P along the axis of an extensible rod: dL = P L / (E A)."""
    n, L, r, E = 8, 0.1, 0.01, 1e6
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, 0), damp=1000.0)
    P = 0.5
    f = np.zeros((n + 1, 3))
    f[-1, 0] = P                                           # rod lies along +x
    spec = spec.replace(f_ext=f)
    spec = spec.replace(dt=oracle.Rod(spec).dt_rule())
    s = _relax(oracle, spec, st, 200000, chunk=2000, tol=1e-14)
    dL = s.x[-1, 0] - L
    assert abs(dL / (P * L / (E * math.pi * r * r)) - 1) < 1e-6


def test_torsion_closed_form(oracle):
    """Static tip torque T about the rod axis: twist over the frame span = T (L - l) / (G J)."""
    n, L, r, E, nu = 8, 0.2, 0.01, 1e6, 0.5
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, 0), damp=0.0)
    G, J = E / (2 * (1 + nu)), math.pi * r ** 4 / 2
    T = 1e-4
    tq = np.zeros((n, 3))
    tq[-1, 2] = T                                          # body axis 3 = rod tangent
    spec = spec.replace(tau_ext=tq, damp_ang=400.0, damp_lin=400.0)
    spec = spec.replace(dt=oracle.Rod(spec).dt_rule())
    s = _relax(oracle, spec, st, 400000, chunk=4000, tol=1e-15)
    rel = oracle.qmul(s.q[0] * np.array([1, -1, -1, -1]), s.q[-1])
    phi = 2 * math.atan2(np.linalg.norm(rel[1:]), rel[0])
    ref = T * (L - L / n) / (G * J)
    assert abs(phi / ref - 1) < 2e-3                       # small-angle (sin) nonlinearity only


def _cantilever(oracle, n, load, L=1.0, r=0.01, E=1e10, rho=1000.0):
    A, I = math.pi * r * r, math.pi * r ** 4 / 4
    omega1 = 1.875 ** 2 * math.sqrt(E * I / (rho * A * L ** 4))
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, 0), damp=2 * omega1)
    if load == "weight":
        spec = spec.replace(gravity=(0, 0, -9.81))
    else:
        f = np.zeros((n + 1, 3))
        f[-1, 2] = -load
        spec = spec.replace(f_ext=f)
    spec = spec.replace(dt=oracle.Rod(spec).dt_rule())
    s = _relax(oracle, spec, st, 600000, chunk=5000, tol=1e-11)
    return -s.x[-1, 2]


@pytest.mark.slow
def test_euler_bernoulli_cantilever(oracle):
    """Small-deflection cantilever under its own weight and under a tip load.

    Frame 0 is clamped and the first joint sits at point 1, so the first half element is
    rigid: the discrete rod is an Euler-Bernoulli cantilever of free length L - l/2 carrying
    the load of the whole length, tip sag w (L - l/2)^4 / (8 E I) for the weight w = rho A g
    and P (L - l/2)^3 / (3 E I) for a tip load P.  The remaining differences (lumping
    O(1/N^2), shear O(E I / (G A L^2)), geometric nonlinearity O((sag / L)^2)) stay within
    1 %; against the plain closed forms the error is first order, about 2 / N."""
    L, r, E, rho = 1.0, 0.01, 1e10, 1000.0
    A, I = math.pi * r * r, math.pi * r ** 4 / 4
    w = rho * A * 9.81
    errs = {}
    for n in (16, 32):
        le = L - 0.5 * L / n
        sag = _cantilever(oracle, n, "weight")
        assert abs(sag / (w * le ** 4 / (8 * E * I)) - 1) < 0.01
        errs[n] = 1 - sag / (w * L ** 4 / (8 * E * I))
    assert 1.7 < errs[16] / errs[32] < 2.3                 # converges like 1/N
    P = 0.05
    le = L - 0.5 * L / 32
    tip = _cantilever(oracle, 32, P)
    assert abs(tip / (P * le ** 3 / (3 * E * I)) - 1) < 0.01


@pytest.mark.slow
def test_first_bending_frequency(oracle):
    """Undamped cantilever under gravity oscillates about its static sag at
    f1 = (1.875^2 / 2 pi) sqrt(E I / (rho A L_e^4)) within 2 %, with the free length
    L_e = L - l/2 of the discrete clamp."""
    n, L, r, E, rho = 24, 1.0, 0.01, 1e10, 1000.0
    A, I = math.pi * r * r, math.pi * r ** 4 / 4
    le = L - 0.5 * L / n
    f1 = 1.875 ** 2 / (2 * math.pi) * math.sqrt(E * I / (rho * A * le ** 4))
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, -9.81), damp=0.0)
    dt = oracle.Rod(spec).dt_rule()
    spec = spec.replace(dt=dt)
    n_steps = int(3.2 / f1 / dt)
    _, tip = oracle.Rod(spec).rollout(st, n_steps, tip=True)
    z = tip[:, 2] - 0.5 * (tip[:, 2].max() + tip[:, 2].min())
    up = np.where((z[:-1] < 0) & (z[1:] >= 0))[0]
    assert len(up) >= 3
    period = (up[-1] - up[0]) * dt / (len(up) - 1)
    assert abs(1.0 / period / f1 - 1) < 0.02


def test_energy_error_is_bounded_and_first_order(oracle):
    """Symplectic Euler, extensible, gamma = 0, a rod falling and swinging under gravity:
    the total energy error stays in a band well below the kinetic-energy scale and the band
    halves when dt halves (first-order, bounded, no secular growth)."""
    spec, st = W.straight_rod(12, L=0.5, gravity=(0, 0, -9.81), damp=0.0)
    dt = oracle.Rod(spec).dt_rule()
    bands = []
    for div in (1, 2):
        rod = oracle.Rod(spec.replace(dt=dt / div))
        E0 = rod.energy(st.x, st.q)
        s, E, K = st, [], []
        for k in range(200):
            s, _ = rod.rollout(s, 500 * div)
            E.append(rod.energy(s.x, s.q) + rod.kinetic(s.v, s.w) - E0)
            K.append(rod.kinetic(s.v, s.w))
        E = np.array(E)
        assert np.isfinite(E).all()
        bands.append(np.abs(E).max())
        assert bands[-1] < 0.25 * max(K)
    assert 1.6 < bands[0] / bands[1] < 2.6


def test_dt_rule_is_stable_and_not_vacuous(oracle):
    """The stability rule's dt runs without blow-up (finite, strains < 50 %, energy never above
    2 E_0) on the c0 rod and on 16 rods of the batched workload, and is within a factor 4 of
    the blow-up limit on c0 (at 4 x the rule the c0 run does blow up)."""
    wl = W.config0(dt=1e-6)
    spec, st = wl.rods[0]
    rule = oracle.Rod(spec).dt_rule()
    assert oracle.Rod(spec.replace(dt=rule)).stable(st, 2000, energy_factor=2.0)
    assert not oracle.Rod(spec.replace(dt=4 * rule)).stable(st, 2000, energy_factor=2.0)
    wl3 = W.config3(n_rods=64, n_min=32, n_max=128)
    for spec, st in wl3.rods[:16]:
        rule = oracle.Rod(spec.replace(dt=1.0)).dt_rule()
        assert oracle.Rod(spec.replace(dt=rule)).stable(st, 1000, energy_factor=2.0)


def test_dt_golden_is_reproducible(oracle):
    """The stored c0 time step is half the bisected largest stable dt of the oracle."""
    g = W.load_dt_golden()["c0"]
    wl = W.config0(dt=1e-6)
    spec, st = wl.rods[0]
    dmax = g["dt_max"]
    assert oracle.Rod(spec.replace(dt=dmax)).stable(st, 2000)
    assert not oracle.Rod(spec.replace(dt=dmax * 1.002)).stable(st, 2000)
    assert g["dt"] == 0.5 * dmax


def test_timoshenko_shear_term_pins_penalty_stiffness(oracle):
    """A soft penalty (K_p = kp G A) acts as shear compliance: a tip load P deflects the
    cantilever by P L_e^3 / (3 E I) + P L / K_p (Timoshenko), within 1 %."""
    n, L, r, E, nu = 16, 1.0, 0.01, 1e10, 0.5
    A, I, G = math.pi * r * r, math.pi * r ** 4 / 4, E / (2 * (1 + nu))
    kp = 1e-4
    omega1 = 1.875 ** 2 * math.sqrt(E * I / (1000.0 * A * L ** 4))
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, 0), damp=2 * omega1)
    P = 0.02
    f = np.zeros((n + 1, 3))
    f[-1, 2] = -P
    spec = spec.replace(f_ext=f, kp_scale=kp)
    spec = spec.replace(dt=oracle.Rod(spec).dt_rule())
    s = _relax(oracle, spec, st, 600000, chunk=5000, tol=1e-12)
    le = L - 0.5 * L / n
    ref = P * le ** 3 / (3 * E * I) + P * L / (kp * G * A)
    assert abs(-s.x[-1, 2] / ref - 1) < 0.01


def test_torsional_frequency(oracle):
    """Constant tip torque switched on at rest: the twist oscillates at the first torsional
    frequency of a clamped-free shaft, f = sqrt(G / rho) / (4 L_e), within 2 %."""
    n, L, r, E, nu, rho = 24, 1.0, 0.01, 1e6, 0.5, 1000.0
    G = E / (2 * (1 + nu))
    spec, st = W.straight_rod(n, L=L, radius=r, young=E, gravity=(0, 0, 0), damp=0.0)
    tq = np.zeros((n, 3))
    tq[-1, 2] = 1e-6
    spec = spec.replace(tau_ext=tq)
    dt = oracle.Rod(spec).dt_rule()
    spec = spec.replace(dt=dt)
    le = L - 0.5 * L / n
    f = math.sqrt(G / rho) / (4 * le)
    rod = oracle.Rod(spec)
    s, phis = st, []
    n_chunk = max(1, int(0.02 / f / dt))
    for k in range(int(3.3 / f / dt / n_chunk)):
        s, _ = rod.rollout(s, n_chunk)
        rel = oracle.qmul(s.q[0] * np.array([1, -1, -1, -1]), s.q[-1])
        phis.append(2 * math.atan2(rel[3], rel[0]))   # twist about body axis 3
    z = np.array(phis) - 0.5 * (max(phis) + min(phis))
    up = np.where((z[:-1] < 0) & (z[1:] >= 0))[0]
    assert len(up) >= 3
    period = (up[-1] - up[0]) * n_chunk * dt / (len(up) - 1)
    assert abs(1.0 / period / f - 1) < 0.02


def test_impulses_conserve_momentum_and_spare_the_clamp(oracle):
    """Constraint impulses are internal: with no other forces the total linear momentum of a
    free chain is unchanged (inverse-mass weighting), and a clamped point never moves."""
    rng = np.random.default_rng(24)
    n, L, r, rho = 9, 0.9, 0.01, 1000.0
    spec, st = W.straight_rod(n, L=L, radius=r, inextensible=True, gravity=(0, 0, 0),
                              dt=1e-3, n_iter=50, clamp=False)
    spec = spec.replace(kp_scale=0.0, bend_scale=0.0, twist_scale=0.0,
                        seg_len=rng.uniform(0.08, 0.12, n), radius=rng.uniform(0.005, 0.02, n))
    x = np.zeros((n + 1, 3))
    x[1:, 0] = np.cumsum(spec.seg_len)
    st.x = x
    st.v = rng.normal(0, 0.5, size=st.v.shape)
    m = rho * math.pi * spec.radius ** 2 * spec.seg_len
    M = np.zeros(n + 1)
    M[:-1] += 0.5 * m
    M[1:] += 0.5 * m
    out, _ = oracle.Rod(spec).rollout(st, 1)
    p0, p1 = (M[:, None] * st.v).sum(0), (M[:, None] * out.v).sum(0)
    assert np.abs(p1 - p0).max() < 1e-13 * np.abs(M[:, None] * st.v).sum()
    spec_c = spec.replace(clamp=True, clamp_x0=tuple(x[0]), clamp_q0=tuple(st.q[0]))
    out, _ = oracle.Rod(spec_c).rollout(st, 3)
    assert np.array_equal(out.x[0], x[0])


def test_velocity_damping_decay(oracle):
    """gamma is plain velocity damping: a free rod translating rigidly and spinning about its
    own axis (no strain) loses speed exactly as (1 - gamma dt)^k."""
    n, gam, dt, k = 6, 3.0, 1e-3, 200
    spec, st = W.straight_rod(n, L=0.3, gravity=(0, 0, 0), damp=gam, dt=dt, clamp=False)
    st.v[:] = [0.2, -0.1, 0.3]
    st.w[:, 2] = 5.0
    out, _ = oracle.Rod(spec).rollout(st, k)
    fac = (1 - gam * dt) ** k
    assert np.allclose(out.v, st.v * fac, rtol=1e-10, atol=0)
    assert np.allclose(out.w[:, 2], 5.0 * fac, rtol=1e-10)


def test_free_rigid_body_keeps_world_angular_momentum(oracle):
    """A single frame with no coupling is a torque-free rigid body: Euler's equations with the
    gyroscopic term keep the world angular momentum R I w fixed (to the method's O(dt))."""
    spec, st = W.straight_rod(1, L=0.05, radius=0.01, gravity=(0, 0, 0), damp=0.0, clamp=False)
    spec = spec.replace(kp_scale=0.0)
    r, l, m = 0.01, 0.05, 1000.0 * math.pi * 0.01 ** 2 * 0.05
    Idiag = np.array([m * (3 * r * r + l * l) / 12] * 2 + [m * r * r / 2])
    st.w[0] = [3.0, -2.0, 40.0]
    drift = []
    for dt in (2e-5, 1e-5):
        out, _ = oracle.Rod(spec.replace(dt=dt)).rollout(st, int(0.05 / dt))
        Lw0 = oracle.rotmat(st.q[0]) @ (Idiag * st.w[0])
        Lw1 = oracle.rotmat(out.q[0]) @ (Idiag * out.w[0])
        drift.append(np.linalg.norm(Lw1 - Lw0) / np.linalg.norm(Lw0))
    assert drift[1] < 5e-3 and 1.6 < drift[0] / drift[1] < 2.5
    # the same motion without the gyroscopic coupling would precess visibly
    assert np.abs(out.w[0, :2] - st.w[0, :2]).max() > 1.0


def test_intrinsic_curvature_rest_shape(oracle):
    """With u_hat = kappa e_1 on every joint and no load the rod relaxes to u = u_hat: frames
    turn about d_1 by 2 asin(kappa l / 2) per joint and the points lie on a circle of radius
    1 / kappa through the clamp, bending towards -d_2."""
    n, L, kappa = 20, 0.5, 2.0
    spec, st = W.straight_rod(n, L=L, gravity=(0, 0, 0), damp=30.0)
    uh = np.zeros((n - 1, 3))
    uh[:, 0] = kappa
    spec = spec.replace(u_hat=uh)
    spec = spec.replace(dt=oracle.Rod(spec).dt_rule())
    s = _relax(oracle, spec, st, 600000, chunk=5000, tol=1e-13)
    rod = oracle.Rod(spec)
    for j in range(n - 1):
        assert np.allclose(rod.darboux(s.q, j), [kappa, 0, 0], atol=1e-6)
    # circle through x_0, tangent +x there, centre on the -y side (d_2 = +y for this clamp)
    Rc = 1.0 / kappa
    l = L / n
    centre = np.array([l / 2, -math.sqrt(Rc * Rc - l * l / 4), 0.0])
    d = np.linalg.norm(s.x - centre, axis=1)
    assert np.abs(d - Rc).max() < 1e-6
    assert s.x[-1, 1] < -0.1


def test_clamp_follows_prescribed_motion(oracle):
    spec, st = W.straight_rod(5, L=0.2, gravity=(0, 0, -9.81), damp=0.1, dt=1e-4)
    spec = spec.replace(clamp_amp=(0.0, 0.002, 0.001), clamp_twist_amp=0.1, clamp_freq=20.0,
                        clamp_phase_x=0.3, clamp_phase_twist=0.7, clamp_twist_axis=(1, 0, 0))
    rod = oracle.Rod(spec)
    xc, qc, _ = rod.clamp_pose(0.0)
    st.x = st.x - st.x[0] + xc
    st.q[0] = qc
    out, _ = rod.rollout(st, 37)
    xc, qc, wc = rod.clamp_pose(37 * spec.dt)
    assert np.allclose(out.x[0], xc, atol=1e-15) and np.allclose(out.q[0], qc, atol=1e-15)
    assert np.allclose(out.w[0], wc, atol=1e-12)
