"""Continuous-batching server (GPU): requests arriving while others run are
admitted as slots and HBM budget free up, and every result equals the same
lattice run alone (bit for bit)."""
import numpy as np
import pytest

import oracle
from paper_1909_04166_amd import lb, serve, workloads as W

pytestmark = pytest.mark.gpu


def _requests():
    reqs = []
    # 51280 nodes in total against a budget of 40000: the late ones must wait
    specs = [(96, 1.2, 300, 0.00), (64, 1.4, 120, 0.00), (128, 1.1, 200, 0.00),
             (80, 1.3, 90, 0.00), (72, 1.5, 260, 0.00), (100, 1.25, 150, 0.02)]
    for i, (n, asp, steps, t) in enumerate(specs):
        case, phi0 = W.ellipse(n, asp)
        reqs.append(serve.Request(rid=i, case=case, phi0=phi0, steps=steps, arrival=t,
                                  want_fields=True))
    return reqs


def test_served_results_equal_alone_runs():
    reqs = _requests()
    # budget for ~3 of these lattices at once: later arrivals must wait
    S = serve.Server(slots=4, node_capacity=40000, precision="fp32", tick=32)
    stats = S.run(reqs)
    print("   serve stats", stats, flush=True)
    assert stats["failed"] == 0 and stats["requests"] == len(reqs)
    waited = [r for r in S.finished if r.admitted - r.arrival > 1e-3]
    assert waited, "the budget should have made some request wait"
    for r in S.finished:
        L = lb.Lattice(r.case, r.phi0, "fp32")
        L.step(r.steps)
        for u, v in zip(r.fields, L.fields()):
            assert np.array_equal(u, v, equal_nan=True)
        assert r.diag["step"] == r.steps
        # and against the FP64 oracle: FP32 phi within 1e-4, p and u within 1e-3
        # of their scale (Laplace pressure sigma / R_eq, capillary velocity sigma / mu_A)
        o = oracle.Oracle(r.case, r.phi0)
        o.step(r.steps)
        fo = o.fields()
        sig = r.case["sigma0"]
        ps = max(np.abs(fo[1]).max(), sig / 12.0)
        us = max(np.abs(fo[2]).max(), np.abs(fo[3]).max(), sig / (r.case["rho_A"] * r.case["nu_A"]))
        e_phi = np.abs(r.fields[0] - fo[0]).max()
        e_p = np.abs(r.fields[1] - fo[1]).max() / ps
        e_u = max(np.abs(r.fields[2] - fo[2]).max(), np.abs(r.fields[3] - fo[3]).max()) / us
        print(f"   request {r.rid} ({r.steps} steps) vs oracle: phi {e_phi:.2e} p {e_p:.2e} u {e_u:.2e}",
              flush=True)
        assert e_phi <= 1e-4 and e_p <= 1e-3 and e_u <= 1e-3
    S.close()


def test_oversize_request_is_refused_not_crashing():
    S = serve.Server(slots=2, node_capacity=10000, precision="fp32")
    case, phi0 = W.ellipse(128, 1.2)
    r = serve.Request(rid=0, case=case, phi0=phi0, steps=10)
    stats = S.run([r])
    assert stats["failed"] == 1 and r.error is not None
    S.close()
