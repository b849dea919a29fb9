"""The cascaded pair with the printed closed forms of the hydrodynamic moment
changes h_3..h_8 (collision "printed", the other reading of Sec. 4 kept as an
option), GPU through the C-ABI against the oracle's printed cascade."""
import numpy as np
import pytest

import oracle
from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tile", [(64, 16), (260, 40), (516, 24)])
@pytest.mark.parametrize("shape,bc,st,seed", [
    ((130, 66), "periodic", "geometric", 1),
    ((100, 72), "wall", "geometric", 2),
    ((200, 40), "wall", "chempot", 3),
])
def test_printed_random_cases_fp64(tile, shape, bc, st, seed):
    nx, ny = shape
    case, phi0 = W.random_case(nx, ny, seed=seed, bc_y=bc, st_form=st, collision="printed")
    if bc == "wall":
        case.update(gy=-2e-5)
    print(f"[case] printed {nx}x{ny} {bc} {st} tile {tile}", flush=True)
    g = lb.Lattice(case, phi0, "fp64", tile=tile)
    o = oracle.Oracle(case, phi0)
    g.step(60)
    o.step(60)
    fg, gg = g.get_dist()
    fo, go = o.get_dist()
    assert np.abs(fg - fo).max() <= 1e-10
    assert np.abs(gg - go).max() <= 1e-10 * max(1.0, np.abs(go).max())


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("fp16", 5e-3)])
def test_printed_droplet_reduced_precision(prec, tol):
    case, phi0 = W.droplet(100, 20.0, W=5.0, ratio=10.0, ny=90)
    case["collision"] = "printed"
    print(f"[case] printed droplet {prec}", flush=True)
    g = lb.Lattice(case, phi0, prec)
    o = oracle.Oracle(case, phi0)
    g.step(100)
    o.step(100)
    err = np.abs(g.fields()[0] - o.fields()[0]).max()
    print(f"   phi error {err:.2e}", flush=True)
    assert err <= tol


def test_printed_batch_equals_single():
    cases = [W.droplet(96, 20.0, ratio=100.0), W.rayleigh_taylor(72, 200, ratio=3.0, Re=256.0)]
    for c, _ in cases:
        c["collision"] = "printed"
    B = lb.Batch(4, 40000, "fp32")
    slots = [B.add(c, p) for c, p in cases]
    B.step(33)
    for s, (c, p) in zip(slots, cases):
        L = lb.Lattice(c, p, "fp32")
        L.step(33)
        for u, v in zip(B.fields(s), L.fields()):
            assert np.array_equal(u, v, equal_nan=True)
