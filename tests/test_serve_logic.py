"""Host logic of the continuous-batching server (CPU, with a stand-in for the
device batch): admission within the slot and node budget, FIFO order with
skip-ahead for requests that fit, results taken at exactly the requested step,
refusal of requests larger than the budget, and cancellation of queued and
resident requests."""
import numpy as np

from paper_1909_04166_amd import serve


class FakeBatch:
    """Counts steps per occupied slot; no device work."""

    def __init__(self, slots):
        self.free = list(range(slots))
        self.steps = {}
        self.log = []

    def add(self, case, phi0):
        s = self.free.pop(0)
        self.steps[s] = 0
        self.log.append(("add", s))
        return s

    def remove(self, slot):
        del self.steps[slot]
        self.free.append(slot)
        self.log.append(("remove", slot))

    def step(self, n, use_graph=True):
        assert n >= 1
        for s in self.steps:
            self.steps[s] += n

    def t(self, slot):
        return self.steps[slot]

    def diagnostics(self, slot):
        return {"step": float(self.steps[slot]), "nan_flag": 0.0}

    def fields(self, slot):
        return (np.zeros(1),) * 4


def _server(slots, capacity, tick=10):
    S = serve.Server.__new__(serve.Server)
    S.batch = FakeBatch(slots)
    S.precision, S.slots, S.capacity, S.tick = "fp32", slots, capacity, tick
    S.queue, S.active, S.finished = serve.collections.deque(), {}, []
    t = [0.0]

    def clock():
        t[0] += 1e-3
        return t[0]
    S.clock = clock
    S.t0 = 0.0
    return S


def _req(rid, n, steps):
    return serve.Request(rid=rid, case={"nx": n, "ny": n}, phi0=np.zeros((n, n)), steps=steps)


def test_budget_fifo_and_exact_steps():
    S = _server(slots=3, capacity=2 * 64 * 64 + 1100)  # room for a 32^2 request, not a 64^2 one
    reqs = [_req(0, 64, 35), _req(1, 64, 12), _req(2, 64, 50), _req(3, 32, 7)]
    stats = S.run(reqs)
    assert stats["failed"] == 0 and stats["requests"] == 4
    for r in S.finished:
        assert r.diag["step"] == r.steps  # ticks never overshoot a resident request
    # request 2 had to wait for a retirement; request 3 (small) skipped ahead of it
    r = {q.rid: q for q in S.finished}
    assert r[3].admitted < r[2].admitted
    assert r[2].admitted >= r[1].done
    assert S.active == {} and sorted(S.batch.free) == [0, 1, 2]


def test_oversize_request_refused():
    S = _server(slots=2, capacity=1000)
    big, small = _req(0, 64, 10), _req(1, 16, 10)
    stats = S.run([big, small])
    assert big.error is not None and small.error is None
    assert stats["failed"] == 1


def test_cancel_queued_and_resident():
    S = _server(slots=1, capacity=10 ** 6, tick=5)
    a, b, c = _req(0, 32, 40), _req(1, 32, 30), _req(2, 32, 20)
    state = {"ticks": 0}

    def on_tick(srv):
        state["ticks"] += 1
        if state["ticks"] == 1:
            assert srv.cancel(1)           # still queued behind a
            assert srv.cancel(0)           # resident: its slot is freed at once
            assert not srv.cancel(0)       # already gone
    S.run([a, b, c], on_tick=on_tick)
    assert a.error == "cancelled" and b.error == "cancelled" and c.error is None
    assert c.diag["step"] == 20
    assert ("remove", 0) in S.batch.log and S.active == {}
