"""Host logic of bench.py (CPU): the kernel-code fingerprint that guards the
counter-measured traffic, when that traffic applies, the request stream of the
served benchmark, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_code_only_ignores_comments_and_blank_lines():
    a = "int x = 1;  // one\n\n/* block\n comment */\nint y = x + 2;\n"
    b = "int x = 1;\n// another remark\nint y = x + 2;   \n"
    c = "int x = 1;\nint y = x + 3;\n"
    assert bench._code_only(a, False) == bench._code_only(b, False)
    assert bench._code_only(a, False) != bench._code_only(c, False)
    p1 = "x = 1  # note\n\ny = 2\n"
    p2 = "# header\nx = 1\ny = 2\n"
    assert bench._code_only(p1, True) == bench._code_only(p2, True)


def test_traffic_table_matches_the_kernel_code():
    """The committed counter passes were taken on the committed kernels; after a
    change to the kernel code they must be taken again (otherwise the benchmark
    reports traffic as null)."""
    assert bench.kernel_fingerprint() == bench.TRAFFIC["fingerprint"]


def test_measured_traffic_applies_to_its_schedule_only():
    rec = bench.TRAFFIC["fp64"]
    tile = rec["tile"]
    assert bench.measured_traffic("tiled8192", "fp64", tile) == rec
    other = list(tile)
    other[1] += 1
    assert bench.measured_traffic("tiled8192", "fp64", other) is None
    assert bench.measured_traffic("tiled4096", "fp64", tile) is None
    assert bench.measured_traffic("tiled8192", "bf16", tile) is None
    assert rec["read"] >= 18 * 8 * 8192 * 8192 and rec["write"] >= 18 * 8 * 8192 * 8192


def test_served_requests_are_seeded():
    a = bench.served_requests(40, 50.0, seed=5)
    b = bench.served_requests(40, 50.0, seed=5)
    assert [(r.case["nx"], r.steps, r.arrival) for r in a] == [(r.case["nx"], r.steps, r.arrival) for r in b]
    t = [r.arrival for r in a]
    assert all(x <= y for x, y in zip(t, t[1:]))
    assert all(64 <= r.case["nx"] == r.case["ny"] <= 1024 for r in a)
    assert all(500 <= r.steps <= 20000 for r in a)


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stdout + out.stderr
