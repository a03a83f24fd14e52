"""Writes dt_bisect.json: the largest stable time step of workloads c0 and c1, found by the
FP64 oracle (log-space bisection over [1e-9, 1e-1] s to a relative width of 1e-3), and the
step used by the workloads, half of it.

Stability over a run means: every value finite, every segment within 50 % of its rest
length, and total energy never above 1.01 E_0 + 1e-9 J.  c0 is tested over its 2000 steps;
c1 (two 512-element rods) over 2000 steps with the clamps held still, taking the smaller
dt_max of the two rods.

Run:  python tests/golden/make_dt_bisect.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2509_04277_amd import workloads as W  # noqa: E402


def main():
    out = {}
    t = time.time()
    wl = W.config0(dt=1e-6)
    spec, st = wl.rods[0]
    dmax = O.bisect_dt_max(spec, st, wl.n_steps)
    out["c0"] = {"dt_max": dmax, "dt": 0.5 * dmax, "bisect_steps": wl.n_steps}
    print("c0 dt_max %.6e (%.1fs)" % (dmax, time.time() - t), flush=True)
    t = time.time()
    wl = W.config1(dt=1e-8, static_clamp=True)
    dms = [O.bisect_dt_max(spec, st, 2000) for spec, st in wl.rods]
    dmax = min(dms)
    out["c1"] = {"dt_max": dmax, "dt": 0.5 * dmax, "bisect_steps": 2000,
                 "dt_max_per_rod": dms}
    print("c1 dt_max %s (%.1fs)" % (dms, time.time() - t), flush=True)
    with open(os.path.join(HERE, "dt_bisect.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
