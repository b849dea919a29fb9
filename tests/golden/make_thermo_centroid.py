"""Writes tests/golden/thermo512_centroid.json: the centroid y (sum y phi / sum phi)
and the phi = 1/2 crossings of column nx/2 of the thermocapillary workload
(512 x 256, walls in y, drop R = 32 of density ratio 10 at (256, 64),
sigma(y) = 0.01 - 5e-5 (y - 64), W 4, M 0.02) from the FP64 CPU oracle every 1000
steps up to 50000.  Calls only oracle/ and the seeded workload generator.

    OMP_NUM_THREADS=8 python tests/golden/make_thermo_centroid.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1909_04166_amd import workloads as W  # noqa: E402


def main(total=50000, every=1000):
    case, phi0 = W.config("thermo512")
    o = oracle.Oracle(case, phi0)
    rows = []
    t0 = time.time()
    for s in range(0, total + 1, every):
        if s:
            o.step(every)
        d = o.diagnostics()
        rows.append({"step": int(d["step"]), "centroid_y": d["centroid_y"], "bottom_y": d["spike_y"],
                     "sum_phi": d["sum_phi"], "max_u": d["max_u"]})
        print(f"{s:6d} centroid {d['centroid_y']:.5f} bottom {d['spike_y']:.4f} max_u {d['max_u']:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "thermo512", "case": case, "every": every, "rows": rows,
           "source": "FP64 CPU oracle (oracle/lb_oracle.c)"}
    with open(os.path.join(HERE, "thermo512_centroid.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
