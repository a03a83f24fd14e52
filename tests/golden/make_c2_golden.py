"""Writes c2_oracle_<N>_<variant>.npz: the FP64 oracle's state of the long-rod workload (one
curved rod of N elements, static clamp, 5000 steps) for N = 16384 and 65536, inextensible and
extensible, 10 steps before the end and at the end, on 32 pieces of 8 consecutive elements
(9 points, 8 frames) spread along the rod, the last one ending at the tip; plus the largest
displacement of any point over the run (the position bar's scale).  The rollouts start from
the initial state rounded to FP32, the values the GPU receives.

Run:  python tests/golden/make_c2_golden.py      (a few minutes: four rollouts in parallel)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2509_04277_amd import workloads as W  # noqa: E402

SIZES = (16384, 65536)
WINDOW = 10        # steps between the two stored states
PIECES, PIECE = 32, 8


def fp32(st):
    """The state rounded to FP32 (kept as doubles): the values the GPU receives."""
    out = st.copy()
    for k in ("x", "v", "q", "w"):
        setattr(out, k, np.asarray(getattr(st, k), dtype=np.float32).astype(np.float64))
    return out


def piece_starts(n):
    return np.unique(np.rint(np.linspace(0, n - PIECE, PIECES)).astype(np.int64))


def path(n, inext):
    return os.path.join(HERE, "c2_oracle_%d_%s.npz" % (n, "inext" if inext else "ext"))


def main():
    cases = [(n, inext) for n in SIZES for inext in (True, False)]
    wls = [W.config2(n, inext) for n, inext in cases]
    rods = [(s, fp32(st)) for s, st in (wl.rods[0] for wl in wls)]
    n_steps = wls[0].n_steps
    dt = rods[0][0].dt
    assert all(wl.n_steps == n_steps and wl.rods[0][0].dt == dt for wl in wls)
    a = O.rollout_many_threads(rods, n_steps - WINDOW, n_threads=len(rods))
    b = O.rollout_many_threads([(s, st) for (s, _), st in zip(rods, a)], WINDOW,
                               n_threads=len(rods), t0=(n_steps - WINDOW) * dt)
    for (n, inext), (spec, st0), sa, sb in zip(cases, rods, a, b):
        p0 = piece_starts(n)
        pts = p0[:, None] + np.arange(PIECE + 1)[None, :]
        frs = p0[:, None] + np.arange(PIECE)[None, :]
        disp = float(np.linalg.norm(sb.x - st0.x, axis=1).max())
        np.savez_compressed(path(n, inext), n=n, inextensible=inext, n_steps=n_steps,
                            window=WINDOW, dt=dt, starts=p0, disp=disp,
                            xa=sa.x[pts], qa=sa.q[frs], xb=sb.x[pts], qb=sb.q[frs])
        print("wrote %s (largest displacement %.3e m)" % (path(n, inext), disp))


if __name__ == "__main__":
    main()
