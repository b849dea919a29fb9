"""lb_step_noalloc (GPU, through the C-ABI): a lattice advanced from its two
caller-owned state buffers, with the library's static scratch only, equals the
same lattice advanced by lb_step through a handle and workspace, bit for bit;
two calls in a row, the second on a smaller lattice in another precision.  In
16-bit storage the step count passed in seeds the stochastic rounding as the
handle's own count does (the fp16 case starts from step 7)."""
import numpy as np
import pytest

from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


def _noalloc_vs_handle(case, phi0, prec, n, tile=(0, 0), pre=0):
    import torch
    L = lb.Lattice(case, phi0, prec)
    L.step(pre)
    ck = L.save()  # 16-byte header, then the 18 stored planes of the current buffer
    payload = np.frombuffer(ck, dtype=np.uint8)[16:]
    used = 18 * case["nx"] * case["ny"] * lb.STORE_BYTES[prec]  # bytes the layout defines
    a = torch.from_numpy(payload.copy()).to("cuda:0")
    b = torch.full_like(a, 0xA5)  # poisoned: every defined byte must be rewritten
    cfg = lb.config_from_case(case, prec, tile=tile)
    stream = torch.cuda.current_stream().cuda_stream
    lb.lb_step_noalloc(cfg, a.data_ptr(), b.data_ptr(), a.numel(), L.t, n, stream)
    torch.cuda.synchronize()
    got = (a if n % 2 == 0 else b).cpu().numpy()[:used]
    L.step(n)
    ref = np.frombuffer(L.save(), dtype=np.uint8)[16:16 + used]
    L.close()
    return got, ref


def test_noalloc_equals_handle_step_twice_second_smaller():
    runs = [
        (W.random_case(300, 180, seed=11, bc_y="wall", gy=-1e-5), "fp64", 37),
        (W.droplet(96, 20.0, ratio=100.0, ny=72), "fp32", 20),
    ]
    for (case, phi0), prec, n in runs:
        print(f"[case] lb_step_noalloc {case['nx']}x{case['ny']} {prec} n={n}", flush=True)
        got, ref = _noalloc_vs_handle(case, phi0, prec, n)
        assert np.array_equal(got, ref)


def test_noalloc_langmuir_and_fp16_pinned_tile():
    case, phi0 = W.surfactant_young(0.0244)
    print("[case] lb_step_noalloc Langmuir 51x201 fp16 tile 128x16, from step 7, n=25", flush=True)
    got, ref = _noalloc_vs_handle(case, phi0, "fp16", 25, tile=(128, 16), pre=7)
    assert np.array_equal(got, ref)


def test_noalloc_fp64_prefetching_516_lanes():
    """The FP64 prefetching kernel at 516 lanes (the one the 8192^2 grid runs) on a
    ragged walled lattice: a partial second strip and a partial last item."""
    case, phi0 = W.random_case(700, 150, seed=12, bc_y="wall", gy=-1e-5)
    print("[case] lb_step_noalloc 700x150 fp64 tile 516x64 prefetching, n=21", flush=True)
    got, ref = _noalloc_vs_handle(case, phi0, "fp64", 21, tile=(516, 64, 1))
    assert np.array_equal(got, ref)
