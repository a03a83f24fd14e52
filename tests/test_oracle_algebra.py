"""Pins of the oracle's quaternion algebra and discrete Darboux vector (Sec. 2.1, eqs. (1), (5), (6)).

The Hamilton product and rotation matrix are pinned to scipy's rotation library (composition
of rotations), the B_k matrices to their defining identities, and the discrete strain of eq. (6)
to the closed form of a uniform relative rotation and to eq. (1) evaluated on a smooth frame
field by finite differences.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation as Rot

from paper_2509_04277_amd import workloads as W


def _sp(q):  # scipy stores quaternions scalar-last
    return Rot.from_quat([q[1], q[2], q[3], q[0]])


def _from_sp(r):
    x, y, z, w = r.as_quat()
    return np.array([w, x, y, z])


def _rand_q(rng):
    q = rng.normal(size=4)
    return q / np.linalg.norm(q)


def test_rotmat_matches_scipy(oracle):
    rng = np.random.default_rng(10)
    for _ in range(50):
        q = _rand_q(rng)
        assert np.allclose(oracle.rotmat(q), _sp(q).as_matrix(), atol=1e-14)


def test_hamilton_product_is_rotation_composition(oracle):
    rng = np.random.default_rng(11)
    for _ in range(50):
        a, b = _rand_q(rng), _rand_q(rng)
        r = oracle.qmul(a, b)
        assert np.allclose(oracle.rotmat(r), _sp(a).as_matrix() @ _sp(b).as_matrix(), atol=1e-14)
        ref = _from_sp(_sp(a) * _sp(b))
        assert np.allclose(r, ref, atol=1e-14) or np.allclose(r, -ref, atol=1e-14)


def test_bmat_identities(oracle):
    rng = np.random.default_rng(12)
    B = [oracle.bmat(k) for k in range(3)]
    for k in range(3):
        assert np.array_equal(B[k].T, -B[k])                     # skew-symmetric
        assert np.array_equal(B[k] @ B[k], -np.eye(4))           # right mult. by a unit pure quaternion
    for _ in range(20):
        q, p = _rand_q(rng), _rand_q(rng)
        qbar = q * np.array([1, -1, -1, -1])
        rel = oracle.qmul(qbar, p)
        for k in range(3):
            ek = np.zeros(4)
            ek[k + 1] = 1.0
            assert np.allclose(B[k] @ q, oracle.qmul(q, ek), atol=1e-15)   # B_k q = q (x) e_k
            assert abs((B[k] @ q) @ p - rel[k + 1]) < 1e-15               # (B_k q).p = (q~ p)_k
            assert abs((B[k] @ q) @ q) < 1e-15                             # left point = midpoint


def _rod_for_frames(q, lbar):
    n = q.shape[0]
    spec, _ = W.straight_rod(n, L=lbar * n)
    return spec


def test_darboux_uniform_relative_rotation(oracle):
    """q_{j+1} = q_j (x) (cos th/2, sin th/2 n)  =>  u = (2/lbar) sin(th/2) n exactly."""
    rng = np.random.default_rng(13)
    for _ in range(20):
        q0 = _rand_q(rng)
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        th = rng.uniform(0.0, 2.5)
        q1 = _from_sp(_sp(q0) * Rot.from_rotvec(th * axis))
        if q1 @ q0 < 0:
            q1 = -q1
        lbar = rng.uniform(0.01, 0.2)
        spec = _rod_for_frames(np.stack([q0, q1]), lbar)
        u = oracle.Rod(spec).darboux(np.stack([q0, q1]), 0)
        assert np.allclose(u, (2.0 / lbar) * np.sin(th / 2) * axis, rtol=0, atol=1e-13 / lbar)


def test_darboux_matches_eq1_on_smooth_frames(oracle):
    """Eq. (1): u0 = 1/2 sum_k d_k x d_k', u = R^T u0.  For the frame field
    R(s) = R0 exp(s [Omega]_x) this is Omega; the discrete eq. (6) must converge to it as O(h^2)."""
    rng = np.random.default_rng(14)
    R0 = Rot.from_quat(rng.normal(size=4))
    Omega = np.array([0.7, -1.3, 2.1])
    s, eps = 0.37, 1e-5
    Rs = lambda s: (R0 * Rot.from_rotvec(s * Omega)).as_matrix()
    dR = (Rs(s + eps) - Rs(s - eps)) / (2 * eps)
    u0 = 0.5 * sum(np.cross(Rs(s)[:, k], dR[:, k]) for k in range(3))
    u_eq1 = Rs(s).T @ u0
    assert np.allclose(u_eq1, Omega, atol=1e-8)
    errs = []
    for h in (0.02, 0.01, 0.005):
        qa = _from_sp(R0 * Rot.from_rotvec((s - h / 2) * Omega))
        qb = _from_sp(R0 * Rot.from_rotvec((s + h / 2) * Omega))
        if qa @ qb < 0:
            qb = -qb
        u = oracle.Rod(_rod_for_frames(np.stack([qa, qb]), h)).darboux(np.stack([qa, qb]), 0)
        errs.append(np.linalg.norm(u - u_eq1))
    assert errs[0] < 1e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5   # second order


def test_clamp_pose_trajectory(oracle):
    """Clamp pose follows the prescribed sinusoids; its body rate matches d/dt of q_c."""
    spec, _ = W.straight_rod(4)
    spec = spec.replace(clamp_x0=(0.1, 0.2, 0.3), clamp_amp=(0.01, 0.0, -0.02),
                        clamp_twist_amp=0.3, clamp_twist_axis=(0.0, 2.0, 0.0), clamp_freq=5.0,
                        clamp_phase_x=0.4, clamp_phase_twist=1.1)
    rod = oracle.Rod(spec)
    t, h = 0.0123, 1e-7
    xc, qc, wc = rod.clamp_pose(t)
    ph = 2 * np.pi * 5.0 * t
    assert np.allclose(xc, [0.1 + 0.01 * np.sin(ph + 0.4), 0.2, 0.3 - 0.02 * np.sin(ph + 0.4)],
                       atol=1e-15)
    psi = 0.3 * np.sin(ph + 1.1)
    ref = _sp(np.array([np.cos(psi / 2), 0, np.sin(psi / 2), 0])) * _sp(np.array(spec.clamp_q0))
    assert np.allclose(_sp(qc).as_matrix(), ref.as_matrix(), atol=1e-14)
    _, qa, _ = rod.clamp_pose(t - h)
    _, qb, _ = rod.clamp_pose(t + h)
    rel = (_sp(qa).inv() * _sp(qb)).as_rotvec() / (2 * h)     # body-frame rate
    assert np.allclose(wc, rel, atol=1e-6)
