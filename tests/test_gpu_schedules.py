"""Every way of spreading a step over workgroups gives the same lattice, bit for
bit (GPU, through the C-ABI): items of fixed rows, balanced persistent runs,
and the strip-aligned persistent cut, pinned with
lb_set_schedule, on a ragged lattice of several strips (the last one 6 columns
wide), with and without walls.  One pinned run is also checked against the
oracle."""
import numpy as np
import pytest

import oracle
from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu

# (tile_x, mode, param, prefetch)
SCHEDULES = [
    (64, 0, 64, 0),
    (132, 0, 16, 0),
    (260, 1, 1, 0),
    (260, 1, 2, 0),
    (132, 2, 1, 0),
    (260, 2, 2, 0),
    (516, 1, 1, 0),
    (260, 2, 1, 1),
    (516, 1, 1, 1),
    (64, 0, 2, 1),
    (132, 0, 4, 0),
    (64, 0, 1, 1),
    (260, 0, 1, 0),
]


def _run(case, phi0, prec, sched, steps):
    L = lb.Lattice(case, phi0, prec)
    L.set_schedule(*sched)
    L.step(steps)
    out = L.fields()
    tile = L.tile
    L.close()
    return out, tile


@pytest.mark.parametrize("prec", ["fp64", "fp16"])
@pytest.mark.parametrize("bc_y", ["periodic", "wall"])
def test_pinned_schedules_bit_identical(prec, bc_y):
    # tall enough that every persistent cut gets bands of at least 8 rows (up to
    # 4 resident 260-lane workgroups per CU: 2 x 4 x 256 / 5 strips -> 408 bands)
    case, phi0 = W.random_case(1030, 3400, seed=31, bc_y=bc_y, gy=-1e-5 if bc_y == "wall" else 0.0)
    print(f"[case] schedules {prec} {bc_y} 1030x3400", flush=True)
    ref, _ = _run(case, phi0, prec, SCHEDULES[0], 12)
    for sched in SCHEDULES[1:]:
        print(f"   schedule {sched}", flush=True)
        got, tile = _run(case, phi0, prec, sched, 12)
        assert tile[0] == sched[0] and tile[3] == sched[3]
        if sched[1] != 0:
            assert tile[2] > 0  # a persistent grid
        for a, b in zip(got, ref):
            assert np.array_equal(a, b, equal_nan=True), sched


def test_pinned_strip_aligned_matches_oracle():
    # one 516-lane workgroup per CU: 256 bands of one strip, 8 or 9 rows each
    case, phi0 = W.random_case(300, 2100, seed=32, bc_y="wall", gy=-2e-5)
    print("[case] strip-aligned schedule vs oracle 300x2100", flush=True)
    g = lb.Lattice(case, phi0, "fp64")
    g.set_schedule(516, 2, 1, 0)
    assert g.tile[2] > 0
    g.step(12)
    o = oracle.Oracle(case, phi0)
    o.step(12)
    fg, gg = g.get_dist()
    fo, go = o.get_dist()
    assert np.abs(fg - fo).max() <= 1e-10
    assert np.abs(gg - go).max() <= 1e-10 * max(1.0, np.abs(go).max())


def test_set_schedule_rejects():
    case, phi0 = W.random_case(300, 40, seed=33)
    L = lb.Lattice(case, phi0, "fp64")
    for bad in [(100, 0, 64, 0),   # not a workgroup width
                (260, 3, 1, 0),    # no such mode
                (260, 0, 0, 0),    # items of no rows
                (260, 1, 5, 0),    # multiplier out of range
                (260, 2, 1, 0)]:   # 40 rows: too few for eight bands of 8
        with pytest.raises(lb.LBError) as e:
            L.set_schedule(*bad)
        assert e.value.code == lb.LB_E_INVALID_ARG, bad
    L.set_schedule(132, 0, 8, 0)  # still usable
    L.step(3)
    assert L.t == 3
    L.close()


def test_pinned_schedule_with_graph_replay_and_repin():
    """A pinned persistent schedule replayed through captured graphs (76 steps:
    two graphs of 32 steps and 12 eager ones), then re-pinned mid-run to another
    mode, gives the same lattice as fixed items all along."""
    case, phi0 = W.random_case(1030, 2600, seed=34)
    print("[case] pinned schedule, graph replay and re-pin 1030x2600 fp32", flush=True)
    ref, _ = _run(case, phi0, "fp32", SCHEDULES[0], 100)
    L = lb.Lattice(case, phi0, "fp32")
    L.set_schedule(132, 2, 1, 0)
    L.step(76)
    L.set_schedule(260, 1, 2, 0)  # drops the captured graphs of the first schedule
    L.step(24)
    got = L.fields()
    L.close()
    for a, b in zip(got, ref):
        assert np.array_equal(a, b, equal_nan=True)
