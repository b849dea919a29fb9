"""Built-in initial phase fields (lb_init_fields / lb_batch_add with phi0 NULL):
computed on the device, they equal the seeded generators' fields (which the
oracle starts from) to rounding, and the lattice then evolves as the oracle's."""
import numpy as np
import pytest

import oracle
from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "droplet": lambda: W.droplet(96, 20.0, W=5.0, ratio=100.0, ny=80),
    "bubble": lambda: W.rising_bubble(nx=64, ny=96, D=24.0, xc=32.0, yc=40.0),
    "tiled droplets": lambda: W.tiled(*W.droplet(40, 9.0, W=5.0), 3, 2),
    "ellipse": lambda: W.ellipse(90, 1.4, ratio=10.0),
    "cylinder": lambda: W.elliptic_cylinder(100.0, 0.05, n=80, a=20.0, b=12.0),
    "rayleigh-taylor": lambda: W.rayleigh_taylor(64, 160, ratio=3.0),
    "flat": lambda: W.flat_interface(8, 64),
    "young": lambda: W.surfactant_young(0.0244),
}


@pytest.mark.parametrize("name", list(CASES))
def test_builtin_field_equals_generator(name):
    """The device evaluates the same signed distance and tanh in another order of
    operations: phi0 agrees to rounding (1e-14, about 50 ulp of 1), and so does the
    initial state f = w phi0, gbar = 0 against the oracle's from the generator's
    field."""
    case, phi0 = CASES[name]()
    print(f"[case] built-in init {name} {case['nx']}x{case['ny']} {case['init']}", flush=True)
    L = lb.Lattice(case, None, "fp64")
    L.init(None)
    phi = L.fields()[0]
    err0 = np.abs(phi - phi0).max()
    print(f"   init phi vs generator {err0:.2e}", flush=True)
    assert err0 <= 1e-14
    fg, gg = L.get_dist()
    fo, go = oracle.Oracle(case, phi0).get_dist()
    assert np.abs(fg - fo).max() <= 1e-14 and not gg.any() and not go.any()


def test_builtin_droplet_evolves_as_oracle():
    """A built-in drop then follows the oracle within the FP64 bound (1e-10) over
    40 steps."""
    case, phi0 = CASES["droplet"]()
    L = lb.Lattice(case, None, "fp64")
    L.init(None)
    L.step(40)
    o = oracle.Oracle(case, phi0)
    o.step(40)
    fg, gg = L.get_dist()
    fo, go = o.get_dist()
    assert np.abs(fg - fo).max() <= 1e-10 and np.abs(gg - go).max() <= 1e-10


def test_builtin_batch_add_and_missing_kind():
    case, phi0 = W.droplet(64, 12.0, W=5.0)
    B = lb.Batch(2, 10000, "fp64")
    s = B.add(case, None)
    B.step(3)
    L = lb.Lattice(case, phi0, "fp64")
    L.step(3)
    assert np.abs(B.fields(s)[0] - L.fields()[0]).max() <= 1e-14
    bare, _ = W.uniform_phase(16, 16)
    with pytest.raises(lb.LBError) as e:
        B.add(bare, None)
    assert e.value.code == lb.LB_E_INVALID_ARG
    M = lb.Lattice(bare, None, "fp64")
    with pytest.raises(lb.LBError):
        M.init(None)
