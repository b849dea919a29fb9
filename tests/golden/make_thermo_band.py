"""Writes tests/golden/thermo512_centroid_band.json: the rounding band of the
centroid trajectory in thermo512_centroid.json.  The FP64 CPU oracle runs the
same workload with its initial f perturbed by one part in 1e16 (seeded normal
factors), and the centroid y is recorded every 1000 steps up to 50000; any two
implementations that round differently separate by about as much as the two
oracle runs do.  Calls only oracle/ and the seeded workload generator.

    OMP_NUM_THREADS=8 python tests/golden/make_thermo_band.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1909_04166_amd import workloads as W  # noqa: E402


def main(total=50000, every=1000, seed=100):
    case, phi0 = W.config("thermo512")
    o = oracle.Oracle(case, phi0)
    f, g = o.get_dist()
    rng = np.random.default_rng(seed)
    o.set_dist(f * (1 + 1e-16 * rng.standard_normal(f.shape)), g, 0)
    rows = []
    t0 = time.time()
    for s in range(0, total + 1, every):
        if s:
            o.step(every)
        d = o.diagnostics()
        rows.append({"step": int(d["step"]), "centroid_y": d["centroid_y"]})
        print(f"{s:6d} centroid {d['centroid_y']:.12f} ({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "thermo512", "perturbation": f"f x (1 + 1e-16 N(0,1)), numpy default_rng({seed})",
           "every": every, "rows": rows, "source": "FP64 CPU oracle (oracle/lb_oracle.c)"}
    with open(os.path.join(HERE, "thermo512_centroid_band.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
