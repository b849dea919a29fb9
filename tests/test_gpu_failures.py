"""Failure detection and race freedom on the GPU (HIP through the C-ABI):

- poisoned destination: the buffer a step writes is filled with NaN beforehand;
  every node must be written (the result equals a clean run bit for bit);
- a NaN injected through a checkpoint is reported as LB_E_UNSTABLE by lb_step;
- a run with every launch blocking (HIP_LAUNCH_BLOCKING=1, in a child process)
  gives the same bits: nothing depends on launch overlap;
- serving: a request cancelled mid-run frees its slot and the other results are
  unchanged; a diverging request is retired with an error while the others finish
  bit-identical to their runs alone."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1909_04166_amd import lb, serve, workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("prec,bcx,bcy", [("fp64", "periodic", "periodic"), ("fp64", "wall", "wall"),
                                          ("fp32", "slip", "wall"), ("fp16", "periodic", "slip")])
def test_poisoned_destination_fully_written(prec, bcx, bcy):
    case, phi0 = W.random_case(150, 70, seed=61, bc_y=bcy)
    case.update(bc_x=bcx, rho_A=20.0, gy=-1e-5 if bcy != "periodic" else 0.0)
    print(f"[case] poisoned destination {prec} bc_x={bcx} bc_y={bcy}", flush=True)
    ref = lb.Lattice(case, phi0, prec, tile=(128, 24))
    ref.step(3)
    f, g = ref.get_dist()
    ref.step(1)
    want = ref.get_dist()
    L = lb.Lattice(case, None, prec, tile=(128, 24))
    nan = np.full_like(f, np.nan)
    L.set_dist(nan, nan, 0)  # buffer A: NaN
    L.step(1)                # buffer B: whatever NaN gives
    L.set_dist(f, g, 3)      # buffer B: the valid state; A still NaN
    L.step(1)                # reads B, writes every node of A
    got = L.get_dist()
    assert not np.isnan(got[0]).any() and not np.isnan(got[1]).any()
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_nan_in_checkpoint_reported_unstable():
    case, phi0 = W.droplet(64, 12.0, ratio=10.0)
    L = lb.Lattice(case, phi0, "fp64", diag_every=10)
    L.step(5)
    st = bytearray(L.save())
    k = 16 + 8 * (9 * 64 * 32 + 40)  # one stored FP64 value in the middle of the lattice
    st[k:k + 8] = np.array([np.nan]).tobytes()
    L.load(bytes(st))
    import torch
    rcs = [L.step(10) for _ in range(3)]
    torch.cuda.synchronize()
    rcs.append(L.step(0))
    print("   step codes", rcs, flush=True)
    assert lb.LB_E_UNSTABLE in rcs
    assert L.diagnostics()["nan_flag"] == 1.0


_CHILD = r'''
import hashlib, sys
sys.path.insert(0, sys.argv[1])
from paper_1909_04166_amd import lb, workloads as W
case, phi0 = W.random_case(300, 90, seed=62, bc_y="wall")
case.update(gy=-1e-5)
L = lb.Lattice(case, phi0, "fp32")
L.step(40)
f, g = L.get_dist()
print(hashlib.sha256(f.tobytes() + g.tobytes()).hexdigest())
'''


def test_blocking_launches_same_bits():
    case, phi0 = W.random_case(300, 90, seed=62, bc_y="wall")
    case.update(gy=-1e-5)
    L = lb.Lattice(case, phi0, "fp32")
    L.step(40)
    f, g = L.get_dist()
    here = hashlib.sha256(f.tobytes() + g.tobytes()).hexdigest()
    env = dict(os.environ, HIP_LAUNCH_BLOCKING="1")
    out = subprocess.run([sys.executable, "-c", _CHILD, ROOT], env=env, capture_output=True, text=True,
                         timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == here


def _alone(r, prec):
    L = lb.Lattice(r.case, r.phi0, prec)
    L.step(r.steps)
    return L.fields()


def test_served_cancel_mid_run():
    specs = [(96, 1.2, 400), (64, 1.4, 150), (80, 1.3, 120), (72, 1.5, 200)]
    reqs = []
    for i, (n, asp, steps) in enumerate(specs):
        case, phi0 = W.ellipse(n, asp)
        reqs.append(serve.Request(rid=i, case=case, phi0=phi0, steps=steps, want_fields=True))
    S = serve.Server(slots=2, node_capacity=10 ** 6, precision="fp32", tick=32)
    ticks = []

    def on_tick(srv):
        ticks.append(1)
        if len(ticks) == 2:
            assert srv.cancel(0)  # resident, 64 of 400 steps done
    S.run(reqs, on_tick=on_tick)
    done = {r.rid: r for r in S.finished}
    assert done[0].error == "cancelled"
    for rid in (1, 2, 3):
        r = done[rid]
        assert r.error is None and r.diag["step"] == r.steps
        for u, v in zip(r.fields, _alone(r, "fp32")):
            assert np.array_equal(u, v, equal_nan=True)
    S.close()


def test_served_diverging_request_retired_others_unaffected():
    """With the printed closed forms of the moment changes (the "printed" option,
    used by every request here: a batch runs one kernel) the 128^2 droplet at W 4,
    M 0.02, ratio 1000 diverges near step 450 (the oracle too); served beside
    stable requests (elliptic drops at W 5) it ends with an error, and they finish
    bit-identical to their runs alone."""
    bad_case, bad_phi = W.config("droplet128")
    bad_case = dict(bad_case, collision="printed")
    reqs = [serve.Request(rid=0, case=bad_case, phi0=bad_phi, steps=700)]
    for i, (n, asp) in enumerate([(96, 1.2), (80, 1.3)], start=1):
        case, phi0 = W.ellipse(n, asp, W=5.0)  # stable at W 5
        case["collision"] = "printed"
        reqs.append(serve.Request(rid=i, case=case, phi0=phi0, steps=700, want_fields=True))
    S = serve.Server(slots=4, node_capacity=10 ** 6, precision="fp64", tick=64)
    stats = S.run(reqs)
    done = {r.rid: r for r in S.finished}
    print("   serve stats", stats, {k: v.error for k, v in done.items()}, flush=True)
    assert done[0].error == "unstable"
    for rid in (1, 2):
        r = done[rid]
        assert r.error is None
        for u, v in zip(r.fields, _alone(r, "fp64")):
            assert np.array_equal(u, v, equal_nan=True)
    S.close()
