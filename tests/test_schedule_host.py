"""Work lists of the step kernels (host logic, CPU): the schedule builder of
csrc/lb_sched.hpp is compiled on its own with g++ and its cuts are checked --
every row of every strip of every lattice collided by exactly one work item,
persistent blocks balanced, and the strip-aligned cut putting the same rows of
neighbouring strips on blocks of one XCD (block b runs on XCD b % 8)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1909_04166_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "lb_sched.hpp"
using namespace cmlb;
// stdin: mode tx th mult resident cus max_items nlat, then inst nx ny per lattice
int main() {
    int mode, tx, th, mult, resident, cus, max_items, nlat;
    while (std::scanf("%d %d %d %d %d %d %d %d", &mode, &tx, &th, &mult, &resident, &cus, &max_items, &nlat) == 8) {
        std::vector<LatShape> lats(nlat);
        for (auto& l : lats)
            if (std::scanf("%d %d %d", &l.inst, &l.nx, &l.ny) != 3) return 1;
        Sched sc;
        sc.mode = mode; sc.tx = tx; sc.th = th; sc.mult = mult;
        std::vector<WorkItem> items;
        const bool ok = plan_schedule(lats, resident, cus, sc, max_items, items);
        std::printf("%d %d %d %d\n", ok ? 1 : 0, sc.grid, sc.rows, sc.n_items);
        for (const auto& it : items) std::printf("%d %d %d %d\n", it.inst, it.x0, it.y0, it.y1);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("sched")
    src = d / "plan.cpp"
    src.write_text(DRIVER)
    exe = d / "plan"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)

    def plan(mode, tx, lats, th=64, mult=1, resident=2, cus=256, max_items=1 << 22):
        req = f"{mode} {tx} {th} {mult} {resident} {cus} {max_items} {len(lats)}\n"
        req += "".join(f"{i} {nx} {ny}\n" for i, nx, ny in lats)
        out = subprocess.run([str(exe)], input=req, capture_output=True, text=True, check=True).stdout.split("\n")
        ok, grid, rows, n = map(int, out[0].split())
        items = [tuple(map(int, l.split())) for l in out[1:1 + n]]
        return dict(ok=bool(ok), grid=grid, rows=rows, items=items)
    return plan


def _check_cover(lats, tx, items):
    """Every row of every strip collided exactly once; strips start at multiples
    of tx - 4 inside the lattice."""
    w = tx - 4
    seen = {}
    shapes = {i: (nx, ny) for i, nx, ny in lats}
    for inst, x0, y0, y1 in items:
        if y1 == y0:
            continue  # padding item
        nx, ny = shapes[inst]
        assert 0 <= y0 < y1 <= ny and x0 % w == 0 and 0 <= x0 < nx
        for y in range(y0, y1):
            key = (inst, x0, y)
            assert key not in seen, f"row collided twice: {key}"
            seen[key] = 1
    expect = sum(((nx + w - 1) // w) * ny for _, nx, ny in lats)
    assert len(seen) == expect


def _blocks(res):
    """Items of persistent block b sit at positions b, b + grid, b + 2 grid, ..."""
    g = res["grid"]
    blocks = [[] for _ in range(g)]
    for j, it in enumerate(res["items"]):
        if it[3] > it[2]:
            blocks[j % g].append(it)
    return blocks


@pytest.mark.parametrize("tx,lats", [
    (64, [(0, 200, 130)]),
    (132, [(0, 8192, 100)]),
    (516, [(0, 1000, 77), (1, 130, 300), (2, 64, 9)]),
])
@pytest.mark.parametrize("th", [8, 32, 256])
def test_items_mode0_cover(planner, tx, lats, th):
    res = planner(0, tx, lats, th=th)
    assert res["ok"]
    assert res["grid"] == len(res["items"])
    _check_cover(lats, tx, res["items"])
    assert max(it[3] - it[2] for it in res["items"]) <= th


@pytest.mark.parametrize("tx,lats,resident,mult", [
    (516, [(0, 8192, 8192)], 1, 1),
    (452, [(0, 8192, 8192)], 2, 1),
    (452, [(0, 8192, 8192)], 2, 2),
    (260, [(0, 1000, 77), (1, 130, 300), (2, 64, 9)], 3, 1),
    (64, [(0, 60, 5)], 4, 2),  # fewer rows than blocks
])
def test_persistent_balanced_cover(planner, tx, lats, resident, mult):
    res = planner(1, tx, lats, mult=mult, resident=resident)
    assert res["ok"]
    _check_cover(lats, tx, res["items"])
    G = mult * resident * 256
    assert 0 < res["grid"] <= G
    sizes = [sum(it[3] - it[2] for it in b) for b in _blocks(res)]
    assert max(sizes) <= res["rows"] and min(sizes) > 0


@pytest.mark.parametrize("tx,nx,ny,resident,mult", [
    (452, 8192, 8192, 2, 1),   # 19 strips: 24 bands, 456 blocks
    (516, 8192, 8192, 1, 1),   # 16 strips: 16 bands
    (260, 8192, 8192, 3, 1),   # 32 strips: 24 bands
    (132, 3000, 1000, 4, 2),
])
def test_strip_aligned_cut(planner, tx, nx, ny, resident, mult):
    lats = [(0, nx, ny)]
    res = planner(2, tx, lats, mult=mult, resident=resident)
    assert res["ok"]
    _check_cover(lats, tx, res["items"])
    w = tx - 4
    nstrips = (nx + w - 1) // w
    G = mult * resident * 256
    assert res["grid"] % nstrips == 0
    bands = res["grid"] // nstrips
    assert bands % 8 == 0 and bands >= 8 and bands == G // nstrips // 8 * 8
    blocks = _blocks(res)
    for b, items in enumerate(blocks):
        assert len(items) == 1  # one segment of one strip
        inst, x0, y0, y1 = items[0]
        assert x0 == (b // bands) * w
        sizes = y1 - y0
        assert ny // bands <= sizes <= ny // bands + 1
        if b + bands < len(blocks):
            # the same rows one strip to the right, on the same XCD
            assert blocks[b + bands][0][2:] == (y0, y1)
            assert blocks[b + bands][0][1] == x0 + w
            assert (b + bands) % 8 == b % 8


def test_strip_aligned_batch_of_equal_heights(planner):
    lats = [(0, 900, 512), (3, 2000, 512), (5, 130, 512)]
    res = planner(2, 260, lats, resident=3)
    assert res["ok"]
    _check_cover(lats, 260, res["items"])
    for items in _blocks(res):
        assert len(items) == 1


@pytest.mark.parametrize("lats,resident", [
    ([(0, 900, 512), (1, 900, 500)], 3),   # heights differ
    ([(0, 8192, 60)], 2),                   # fewer than 8 rows per band
    ([(0, 200000, 8192)], 1),               # more strips than blocks: no 8 bands
])
def test_strip_aligned_rejects(planner, lats, resident):
    assert not planner(2, 260, lats, resident=resident)["ok"]


def test_max_items_enforced(planner):
    lats = [(0, 8192, 8192)]
    assert not planner(0, 64, lats, th=8, max_items=1000)["ok"]
    assert planner(0, 64, lats, th=8)["ok"]



SMALL_DRIVER = r"""
#include <cstdio>
#include "lb_sched.hpp"
using namespace cmlb;
// stdin: nx ny prefetch cus min_rows; stdout: tx th mode pf
int main() {
    int nx, ny, pf, cus, mr;
    while (std::scanf("%d %d %d %d %d", &nx, &ny, &pf, &cus, &mr) == 5) {
        const Sched sc = small_lattice_sched(nx, ny, pf != 0, cus, mr);
        std::printf("%d %d %d %d\n", sc.tx, sc.th, sc.mode, sc.pf);
    }
    return 0;
}
"""


def test_small_lattice_schedule(tmp_path):
    """One item per workgroup; rows per item the largest power of two (<= 256)
    that still gives two items per CU, down to single rows; the width by the
    lattice width; prefetching as asked."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "small.cpp"
    src.write_text(SMALL_DRIVER)
    exe = tmp_path / "small"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    cases = [(nx, ny, pf) for nx in (64, 100, 128, 255, 256, 600, 1024, 8192) for ny in (8, 77, 128, 1024, 8192)
             for pf in (0, 1)]
    req = "".join(f"{nx} {ny} {pf} 256 1\n" for nx, ny, pf in cases)
    out = subprocess.run([str(exe)], input=req, capture_output=True, text=True, check=True).stdout.split("\n")
    for (nx, ny, pf), line in zip(cases, out):
        tx, th, mode, got_pf = map(int, line.split())
        assert mode == 0 and got_pf == pf
        assert tx == (256 if nx >= 1024 else 128 if nx >= 256 else 64)
        strips = -(-nx // (tx - 4))
        items = strips * -(-ny // th)
        assert th in (1, 2, 4, 8, 16, 32, 64, 128, 256)
        assert items >= 512 or th == 1, (nx, ny, th)            # enough items, or single rows
        assert th == 256 or strips * -(-ny // (2 * th)) < 512, (nx, ny, th)  # the largest such
    # the 128^2 droplet: three 60-column strips of single rows
    assert out[cases.index((128, 128, 1))].split() == ["64", "1", "0", "1"]
