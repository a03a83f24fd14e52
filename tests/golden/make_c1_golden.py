"""Writes c1_oracle.json: FP64 oracle tip positions of the two c1 rods every 1000 steps over
the full 20000-step run, plus the state of a few sample points at the end, from the initial
state rounded to FP32 (the values the GPU receives).

Run:  python tests/golden/make_c1_golden.py      (about 20 s)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2509_04277_amd import workloads as W  # noqa: E402


def main():
    wl = W.config1()
    out = {"n_steps": wl.n_steps, "every": 1000, "dt": wl.rods[0][0].dt, "rods": []}
    for spec, st in wl.rods:
        st = st.copy()
        for k in ("x", "v", "q", "w"):
            setattr(st, k, np.asarray(getattr(st, k), dtype=np.float32).astype(np.float64))
        final, tip = O.Rod(spec).rollout(st, wl.n_steps, tip=True)
        sample = [0, 1, 2, 100, 255, 256, 400, spec.n - 1, spec.n]
        out["rods"].append({
            "tip": tip[999::1000].tolist(),
            "sample_points": sample,
            "x": final.x[sample].tolist(), "v": final.v[sample].tolist(),
            "q": final.q[[i for i in sample if i < spec.n]].tolist(),
            "max_strain": O.Rod(spec).max_strain(final.x)})
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
