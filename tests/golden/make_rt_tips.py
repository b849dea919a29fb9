"""Writes tests/golden/rt256_tips.json: spike and bubble tip positions of the
Rayleigh-Taylor workload (256 x 1024, At 0.5, Re 3000, W 4, walls in y) from the
FP64 CPU oracle every 500 steps up to 20000.  Calls only oracle/ and the seeded
workload generator.  Tip definitions: lowest phi = 1/2 crossing on column nx/2
(spike) and highest crossing on column 0 (bubble), linear interpolation in y.

    OMP_NUM_THREADS=8 python tests/golden/make_rt_tips.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1909_04166_amd import workloads as W  # noqa: E402


def main(total=20000, every=500):
    case, phi0 = W.config("rt256")
    o = oracle.Oracle(case, phi0)
    rows = []
    t0 = time.time()
    for s in range(0, total + 1, every):
        if s:
            o.step(every)
        d = o.diagnostics()
        rows.append({"step": int(d["step"]), "spike_y": d["spike_y"], "bubble_y": d["bubble_y"],
                     "sum_phi": d["sum_phi"], "max_u": d["max_u"]})
        print(f"{s:6d} spike {d['spike_y']:.3f} bubble {d['bubble_y']:.3f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = {"workload": "rt256", "case": case, "every": every, "rows": rows,
           "source": "FP64 CPU oracle (oracle/lb_oracle.c)"}
    with open(os.path.join(HERE, "rt256_tips.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
