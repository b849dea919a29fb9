"""Batched persistent step over uneven lattices (GPU, through the C-ABI):
every slot evolves exactly as the same lattice alone (bit for bit), whatever
else shares the launch, with or without graph replay, across adds/removes."""
import numpy as np
import pytest

from paper_1909_04166_amd import lb, workloads as W

pytestmark = pytest.mark.gpu


def _cases():
    return [
        W.droplet(96, 20.0, ratio=100.0),
        W.rayleigh_taylor(72, 200, ratio=3.0, Re=256.0),
        W.random_case(130, 66, seed=7, bc_y="wall", gy=-1e-5),
        W.droplet(64, 12.0, ratio=10.0, ny=100),
        W.thermocapillary(160, 96, R=20.0),
    ]


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
def test_batch_slots_equal_single_lattices(prec):
    cases = _cases()
    print(f"[case] batch of {len(cases)} uneven lattices, {prec}", flush=True)
    B = lb.Batch(8, 80000, prec)
    slots = [B.add(c, p) for c, p in cases]
    B.step(37)
    for s, (c, p) in zip(slots, cases):
        L = lb.Lattice(c, p, prec)
        L.step(37)
        a = B.fields(s)
        b = L.fields()
        for x, y in zip(a, b):
            assert np.array_equal(x, y, equal_nan=True)
        assert B.t(s) == 37


def test_batch_graph_replay_equals_eager_and_mix_order():
    """Graphs are replayed once the lattices have held for 128 steps; replays,
    eager steps and reads interleaved give the eager result."""
    cases = _cases()
    A = lb.Batch(8, 80000, "fp32")
    G = lb.Batch(8, 80000, "fp32")
    sa = [A.add(c, p) for c, p in cases]
    sg = [G.add(c, p) for c, p in reversed(cases)][::-1]  # different slot order
    A.step(300, use_graph=False)
    G.step(128, use_graph=True)  # eager: the work list has just been built
    for _ in range(3):  # one graph of 32 steps and 16 eager ones each time, then a read
        G.step(48, use_graph=True)
        G.fields(sg[0])
    G.step(28, use_graph=False)  # 128 + 3 x 48 + 28 = 300
    for x, y in zip(sa, sg):
        for u, v in zip(A.fields(x), G.fields(y)):
            assert np.array_equal(u, v, equal_nan=True)


def test_batch_add_remove_continuous():
    """Slots freed and refilled between steps; a lattice added late evolves as
    if alone, and the ones already running are not disturbed."""
    cases = _cases()
    B = lb.Batch(3, 40000, "fp32")
    s0 = B.add(*cases[0])
    s1 = B.add(*cases[1])
    B.step(10)
    B.remove(s0)
    s2 = B.add(*cases[3])  # reuses the freed slot / memory
    B.step(21)
    assert B.t(s1) == 31 and B.t(s2) == 21
    for s, (c, p), n in [(s1, cases[1], 31), (s2, cases[3], 21)]:
        L = lb.Lattice(c, p, "fp32")
        L.step(n)
        for u, v in zip(B.fields(s), L.fields()):
            assert np.array_equal(u, v, equal_nan=True)
    used, nodes = B.usage()
    assert used == 2 and nodes == 72 * 200 + 64 * 100


def test_batch_rejects_when_full():
    B = lb.Batch(2, 20000, "fp32")
    B.add(*W.droplet(96, 20.0))
    with pytest.raises(lb.LBError) as e:
        B.add(*W.droplet(128, 25.0))  # 16384 more nodes than the capacity left
    assert e.value.code == lb.LB_E_WORKSPACE
    B.add(*W.droplet(64, 12.0))
    with pytest.raises(lb.LBError) as e:
        B.add(*W.droplet(16, 4.0))  # no free slot
    assert e.value.code == lb.LB_E_WORKSPACE


@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_batch_wall_kernels_follow_membership(prec):
    """A batch of periodic lattices runs the kernels without wall logic; adding
    a walled lattice switches to the general ones and removing it switches
    back. Every lattice still evolves bit for bit as it would alone."""
    per0, per1 = W.droplet(96, 20.0, ratio=100.0), W.droplet(64, 12.0, ratio=10.0, ny=100)
    walled = W.random_case(130, 66, seed=7, bc_y="wall", gy=-1e-5)
    print(f"[case] periodic/walled batch membership, {prec}", flush=True)
    B = lb.Batch(4, 60000, prec)
    s0, s1 = B.add(*per0), B.add(*per1)
    B.step(10)
    sw = B.add(*walled)
    B.step(11, use_graph=False)
    got_w = B.fields(sw)
    B.remove(sw)
    B.step(12)
    for (c, p), s, n in [(per0, s0, 33), (per1, s1, 33)]:
        L = lb.Lattice(c, p, prec)
        L.step(n)
        for u, v in zip(B.fields(s), L.fields()):
            assert np.array_equal(u, v, equal_nan=True)
    L = lb.Lattice(*walled, prec)
    L.step(11)
    for u, v in zip(got_w, L.fields()):
        assert np.array_equal(u, v, equal_nan=True)
