"""The Laplace law on the oracle at the paper's own set-up (Sec. 6.2): a static
drop in a 200 x 200 periodic box, R 30 with sigma 1e-3 at density ratios 10,
100 and 1000, and at ratio 1000 sigma 1e-4, 5e-3 and R 20, 40; interface widths
W 4, 5 and 8.  The oracle's pressure jumps are in tests/golden/laplace_paper.json
(written by make_laplace_paper.py, which calls only oracle/); one case is re-run
here and must reproduce the file, so the file belongs to the oracle as it is.

What pins them, independently of the oracle:
  * Delta p = sigma / R (Sec. 6.2) up to the discrete surface energy: for the
    equilibrium profile phi = 1/2 + 1/2 tanh(2 zeta / W) the isotropic gradient
    stencil along a grid line is the central difference, and 1.5 W sum (dphi)^2
    is below 1 by a W-dependent amount (0.939, 0.960, 0.984 at W 4, 5, 8, computed
    below from the profile); the jump must lie within 2.5 % of sigma / R times
    that factor, and tend to sigma / R as W grows;
  * the jump does not depend on the density ratio or (being linear) on sigma;
  * every case is stable, W 4 at ratio 1000 included (robustness, Sec. 6.2)."""
import json
import os

import numpy as np
import pytest

from paper_1909_04166_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "laplace_paper.json")


def discrete_energy_factor(Wd):
    zeta = np.arange(-200, 201, dtype=float)
    phi = 0.5 + 0.5 * np.tanh(2 * zeta / Wd)
    d = (phi[2:] - phi[:-2]) / 2
    return 1.5 * Wd * float((d * d).sum())


def _rows():
    with open(GOLDEN) as fh:
        return json.load(fh)["rows"]


def _final(r):
    return r["dp_every_1000"][-1] * r["R"] / r["sigma"]


def test_discrete_energy_factor_closed_form_limits():
    f = [discrete_energy_factor(w) for w in (4.0, 5.0, 8.0, 32.0)]
    assert abs(f[0] - 0.9391) < 1e-3 and abs(f[1] - 0.9598) < 1e-3 and abs(f[2] - 0.9837) < 1e-3
    assert f[0] < f[1] < f[2] < f[3] and abs(f[3] - 1.0) < 2e-3


def test_every_paper_case_is_stable():
    rows = _rows()
    assert len(rows) == 21
    assert all(r["stable"] for r in rows), [(r["W"], r["ratio"], r["sigma"], r["R"]) for r in rows if not r["stable"]]


@pytest.mark.parametrize("Wd", [4.0, 5.0, 8.0])
def test_laplace_law_with_discrete_energy(Wd):
    kd = discrete_energy_factor(Wd)
    rows = [r for r in _rows() if r["W"] == Wd]
    vals = {(r["ratio"], r["sigma"], r["R"]): _final(r) for r in rows}
    for k, v in vals.items():
        assert abs(v / kd - 1.0) <= 0.025, (Wd, k, v, kd)
    at30 = [vals[(ratio, 1e-3, 30.0)] for ratio in (10.0, 100.0, 1000.0)]
    assert max(at30) - min(at30) <= 0.01 * max(at30)  # independent of the density ratio
    sig = [vals[(1000.0, s, 30.0)] for s in (1e-4, 1e-3, 5e-3)]
    assert max(sig) - min(sig) <= 0.005 * max(sig)  # linear in sigma


def test_laplace_converges_to_the_law_with_width():
    dev = {}
    for Wd in (4.0, 5.0, 8.0):
        r = [x for x in _rows() if x["W"] == Wd and x["ratio"] == 1000.0 and x["sigma"] == 1e-3 and x["R"] == 30.0][0]
        dev[Wd] = abs(1.0 - _final(r))
    assert dev[4.0] > dev[5.0] > dev[8.0] and dev[8.0] <= 0.02


def test_golden_reproduced_by_the_oracle():
    """W 4 at ratio 1000 (the case the printed closed forms cannot run): the first
    1000 steps of the golden run again, to the last bit."""
    import make_laplace_paper as mk
    case, dp, stable, _ = mk.run(4.0, 1000.0, 1e-3, 30.0, steps=1000, every=1000)
    r = [x for x in _rows() if x["W"] == 4.0 and x["ratio"] == 1000.0 and x["sigma"] == 1e-3 and x["R"] == 30.0][0]
    assert stable and dp[0] == r["dp_every_1000"][0]
