"""Writes tests/golden/laplace_paper.json: the static-drop set-up of Sec. 6.2 run
on the FP64 CPU oracle.  200 x 200 periodic, drop of phase A at the centre,
nu 0.1, M 0.02; R 30 with sigma 1e-3 at density ratios 10, 100 and 1000, and at
ratio 1000 sigma 1e-4 and 5e-3 (R 30) and R 20 and 40 (sigma 1e-3); interface
widths W 4, 5 and 8.  The drop starts at rest with its Laplace pressure already
set (gbar_a = w_a sigma / R phi0, so p = sigma / R phi0, u = 0), which shortens
the start-up pressure oscillation; the equilibrium does not depend on it.  The
pressure jump p(centre) - p(corner) is recorded every 1000 steps to 6000.
Calls only oracle/ and the seeded workload generator.

    OMP_NUM_THREADS=8 python tests/golden/make_laplace_paper.py
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

WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
STEPS, EVERY = 6000, 1000


def specs():
    out = []
    for Wd in (4.0, 5.0, 8.0):
        for ratio in (10.0, 100.0, 1000.0):
            out.append((Wd, ratio, 1e-3, 30.0))
        for sig in (1e-4, 5e-3):
            out.append((Wd, 1000.0, sig, 30.0))
        for R in (20.0, 40.0):
            out.append((Wd, 1000.0, 1e-3, R))
    return out


def run(Wd, ratio, sig, R, steps=STEPS, every=EVERY):
    case, phi0 = W.droplet(200, R, W=Wd, ratio=ratio, sigma=sig)
    o = oracle.Oracle(case, phi0)
    f, _ = o.get_dist()
    o.set_dist(f, WT[:, None, None] * (sig / R * phi0)[None], 0)
    dp, stable = [], True
    while o.t < steps:
        o.step(every)
        d = o.diagnostics()
        dp.append(d["dp_laplace"])
        if d["nan_flag"] or not d["max_u"] < 0.3:
            stable = False
            break
    return case, dp, stable, d["r_eff"]


def main():
    rows = []
    t0 = time.time()
    for Wd, ratio, sig, R in specs():
        case, dp, stable, reff = run(Wd, ratio, sig, R)
        rows.append({"W": Wd, "ratio": ratio, "sigma": sig, "R": R, "stable": stable, "r_eff": reff,
                     "dp_every_1000": dp})
        last = dp[-1] * R / sig if stable else float("nan")
        print(f"W {Wd} ratio {ratio:6.0f} sigma {sig:.0e} R {R:.0f}: dp R / sigma {last:.4f} "
              f"{'stable' if stable else 'UNSTABLE'} ({time.time() - t0:.0f} s)", flush=True)
    out = {"set_up": "Sec. 6.2 static drop, 200 x 200 periodic, nu 0.1, M 0.02, Laplace pressure preset",
           "steps": STEPS, "every": EVERY, "rows": rows, "source": "FP64 CPU oracle (oracle/lb_oracle.c)"}
    with open(os.path.join(HERE, "laplace_paper.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
