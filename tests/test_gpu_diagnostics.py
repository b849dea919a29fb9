"""The GPU's FP64 diagnostics (lb_diagnostics through the C-ABI) on synthetic
states whose answers are worked out by hand: the same states as the oracle's
pins (tests/test_oracle_diagnostics.py), set as post-streaming distributions."""
import math

import numpy as np
import pytest

from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu

import test_oracle_diagnostics as T  # noqa: E402  (the states and their answers)


def _gpu_diag(phi, gbar=None, rho_A=3.0, rho_B=1.0, step=0, nx=T.NX, ny=T.NY):
    case = W.base_case(nx, ny, rho_A=rho_A, rho_B=rho_B, sigma0=0.0)
    L = lb.Lattice(case, None, "fp64")
    f = np.zeros((9, ny, nx))
    f[0] = phi
    g = np.zeros((9, ny, nx)) if gbar is None else gbar
    L.set_dist(f, g, step)
    d = L.diagnostics()
    L.close()
    return d


def test_gpu_tips():
    print("[case] diagnostics: tips", flush=True)
    phi = np.zeros((T.NY, T.NX))
    phi[:, 4] = T._column([10, 40, 70])
    phi[:, 0] = T._column([5, 60, 90])
    phi[:, 3], phi[:, 5] = T._column([20]), T._column([30])
    phi[:, 1], phi[:, 8] = T._column([50]), T._column([80])
    d = _gpu_diag(phi)
    assert abs(d["spike_y"] - (10 + 1 / 3)) <= 1e-12
    assert abs(d["bubble_y"] - (90 + 1 / 3)) <= 1e-12
    d = _gpu_diag(np.full((T.NY, T.NX), 0.25))
    assert math.isnan(d["spike_y"]) and math.isnan(d["bubble_y"])


def test_gpu_centroid_sums_radius_velocity_probe_nan():
    print("[case] diagnostics: centroid, sums, max|u|, dp, nan", flush=True)
    nx, ny = T.NX, T.NY
    phi = np.zeros((ny, nx))
    phi[10:20] = 1.0
    phi[50:60] = 0.5
    d = _gpu_diag(phi, rho_A=7.0, rho_B=2.0, step=123)
    assert d["step"] == 123
    assert abs(d["centroid_y"] - (10 * 14.5 + 5 * 54.5) / 15) <= 1e-12
    assert abs(d["sum_phi"] - 15 * nx) <= 1e-12
    assert abs(d["sum_rho"] - (nx * ny * 2.0 + 15 * nx * 5.0)) <= 1e-9
    assert abs(d["r_eff"] - math.sqrt(15 * nx / math.pi)) <= 1e-12
    g = np.zeros((9, ny, nx))
    g[1, 61, 7], g[2, 61, 7] = 0.03, 0.04
    g[1, 20, 2] = -0.045
    g[4, 80, 6] = 0.0449
    assert abs(_gpu_diag(np.ones((ny, nx)), g)["max_u"] - 0.05) <= 1e-14
    g = np.zeros((9, 14, 9))
    g[0] += 1e-3
    g[0, 7, 4], g[0, 4, 7], g[0, 0, 0] = 4e-3, 9e-3, 2e-3
    assert abs(_gpu_diag(np.ones((14, 9)), g, nx=9, ny=14)["dp_laplace"] - 2e-3) <= 1e-15
    phi = np.full((ny, nx), 0.5)
    phi[30, 2] = np.nan
    assert _gpu_diag(phi)["nan_flag"] == 1.0
    g = np.zeros((9, ny, nx))
    g[1, 3, 1] = np.nan
    g[1, 90, 7] = 0.2
    d = _gpu_diag(np.ones((ny, nx)), g)
    assert d["nan_flag"] == 1.0 and math.isnan(d["max_u"])


def test_bandwidth_probe_variants_move_the_data():
    """Every copy variant copies exactly; the write probe writes each word's index;
    the read probe's XOR of a constant array over an even count of words per lane
    is zero."""
    import torch
    print("[case] bandwidth probe variants, 32 MiB", flush=True)
    n = 32 << 20
    a = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for v in (1, 2, 3, 4):
        b = torch.zeros_like(a)
        lb.lb_bandwidth_probe(b.data_ptr(), a.data_ptr(), n, v, stream)
        torch.cuda.synchronize()
        assert torch.equal(a, b), v
    b = torch.zeros_like(a)
    lb.lb_bandwidth_probe(b.data_ptr(), a.data_ptr(), n, 6, stream)
    torch.cuda.synchronize()
    w = b.view(torch.int32).view(-1, 4)
    assert torch.equal(w[:, 0].cpu(), torch.arange(n // 16, dtype=torch.int32)) and not w[:, 1:].any()
    ones = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    b = torch.ones_like(a)
    lb.lb_bandwidth_probe(b.data_ptr(), ones.data_ptr(), n, 5, stream)
    torch.cuda.synchronize()
    assert not b[: 4096 * 256 * 16].any()
    # row-pattern probes: whole rows of 18 x 8064 two-byte values, each value's
    # lowest bit flipped (16-bit words for 7, 32-bit words for 8), the rest untouched
    used = n // (18 * 8064 * 2) * (18 * 8064 * 2)
    for v, flip in ((7, 1), (8, 1)):
        b = torch.zeros_like(a)
        lb.lb_bandwidth_probe(b.data_ptr(), a.data_ptr(), n, v, stream)
        torch.cuda.synchronize()
        if v == 7:
            want = a[:used].view(torch.int16) ^ flip
            got = b[:used].view(torch.int16)
        else:
            want = a[:used].view(torch.int32) ^ flip
            got = b[:used].view(torch.int32)
        assert torch.equal(got, want), v
        assert not b[used:].any(), v
