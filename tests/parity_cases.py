"""Inputs of the parity configurations that the GPU parity tests and the CPU test of the bars
share (seeded, synthetic; no GPU import)."""
import numpy as np

from paper_2509_04277_amd import workloads as W


def edge_rods(oracle):
    """Ragged rods (N = 1, 2, 3, 65, 130, 200), both variants, clamped (driven) and free,
    external loads, intrinsic shape, non-uniform material, random initial velocities."""
    rng = np.random.default_rng(40)
    rods = []
    for n, inext, clamp in ((1, False, True), (2, True, True), (3, False, False), (65, True, True),
                            (130, False, True), (200, True, False)):
        x, q = W.curved_rod(n, 0.02, rng, sigma=0.2, twist_sigma=0.1)
        spec = W.RodSpec(
            n=n, inextensible=inext, n_iter=7 if inext else 0, clamp=clamp, dt=2e-5,
            gravity=(0.5, -2.0, -9.81), damp_lin=0.3, damp_ang=0.2, poisson=0.35, density=1100.0,
            seg_len=rng.uniform(0.015, 0.025, n), radius=rng.uniform(0.004, 0.006, n),
            young=rng.uniform(2e5, 1e6, n), kp_scale=0.8, bend_scale=1.2, twist_scale=0.9,
            u_hat=rng.normal(0, 1.0, (n - 1, 3)) if n > 1 else None,
            f_ext=rng.normal(0, 1e-3, (n + 1, 3)), tau_ext=rng.normal(0, 1e-5, (n, 3)),
            clamp_x0=tuple(x[0]), clamp_q0=tuple(q[0]),
            clamp_amp=(0.0, 1e-3, 5e-4) if clamp else (0, 0, 0), clamp_twist_amp=0.1 if clamp else 0,
            clamp_twist_axis=(0.2, 0.0, 1.0), clamp_freq=7.0, clamp_phase_x=0.3,
            clamp_phase_twist=1.3)
        st = W.RodState(x, rng.normal(0, 1e-2, (n + 1, 3)), q, rng.normal(0, 0.1, (n, 3)))
        if clamp:
            xc, qc, _ = oracle.Rod(spec).clamp_pose(0.0)
            st.x = st.x - st.x[0] + xc
            st.q[0] = qc
        rods.append((spec, st))
    return rods
