"""Continuous-batching request server over the batch C-ABI.

Requests (a lattice set-up plus a number of steps) arrive over time.  The
server keeps every admitted lattice resident in one device workspace, admits a
queued request as soon as a slot and enough nodes of the HBM budget are free,
and advances all resident lattices together: one tick = one replayed graph of
persistent-kernel steps over every occupied slot.  A tick never runs past the
step count of any resident request, so each result is produced at exactly its
requested step, bit-identical to the same lattice run alone.  Finished requests
are read out (FP64 diagnostics, optionally the fields) and their slot and
memory are reused by the next admission.

The slot pool, node allocator, work-list rebuild, autotuned schedule and graph
replay are in the native library; this module is the admission and retirement
policy.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable

import numpy as np

from paper_1909_04166_amd import lb


@dataclasses.dataclass
class Request:
    rid: int
    case: dict
    phi0: np.ndarray | None
    steps: int
    arrival: float = 0.0          # seconds on the server clock
    want_fields: bool = False
    make: Callable[[], np.ndarray] | None = None  # builds phi0 at admission when phi0 is None
    # filled by the server
    admitted: float | None = None
    done: float | None = None
    slot: int | None = None
    diag: dict | None = None
    fields: tuple | None = None
    error: str | None = None

    @property
    def nodes(self) -> int:
        return int(self.case["nx"]) * int(self.case["ny"])

    @property
    def latency(self) -> float | None:
        return None if self.done is None else self.done - self.arrival


class Server:
    """slots: resident lattices at most; node_capacity: HBM budget in lattice
    nodes (2 x 18 stored values per node plus scratch); tick: steps per graph
    replay when no resident request finishes earlier."""

    def __init__(self, slots: int, node_capacity: int, precision: str = "fp32", tick: int = 64,
                 clock: Callable[[], float] | None = None):
        self.batch = lb.Batch(slots, node_capacity, precision)
        self.precision = precision
        self.slots = slots
        self.capacity = node_capacity
        self.tick = int(tick)
        self.queue: collections.deque[Request] = collections.deque()
        self.active: dict[int, Request] = {}
        self.finished: list[Request] = []
        self.clock = clock or time.perf_counter
        self.t0 = self.clock()

    def now(self) -> float:
        return self.clock() - self.t0

    def used_nodes(self) -> int:
        return sum(r.nodes for r in self.active.values())

    def submit(self, req: Request) -> None:
        if req.nodes > self.capacity:
            req.error = "larger than the HBM budget"
            req.done = self.now()
            self.finished.append(req)
            return
        self.queue.append(req)

    def _admit(self) -> None:
        # FIFO; a request that does not fit yet blocks the ones behind it only
        # while a smaller one cannot fit either (skip-ahead for small requests)
        blocked = []
        while self.queue and len(self.active) < self.slots:
            req = self.queue.popleft()
            if self.used_nodes() + req.nodes > self.capacity:
                blocked.append(req)
                if len(blocked) >= 4:
                    break
                continue
            if req.phi0 is None and req.make is not None:
                req.phi0 = req.make()
            try:
                req.slot = self.batch.add(req.case, req.phi0)
            except lb.LBError as e:
                if e.code == lb.LB_E_WORKSPACE:  # fragmentation: retry after retirements
                    blocked.append(req)
                    break
                req.error = str(e)
                req.done = self.now()
                self.finished.append(req)
                continue
            req.admitted = self.now()
            self.active[req.slot] = req
        for r in reversed(blocked):
            self.queue.appendleft(r)

    def _retire(self) -> None:
        for slot, req in list(self.active.items()):
            if self.batch.t(slot) >= req.steps:
                req.diag = self.batch.diagnostics(slot)
                if req.want_fields:
                    req.fields = self.batch.fields(slot)
                if req.diag["nan_flag"]:
                    req.error = "unstable"
                self.batch.remove(slot)
                del self.active[slot]
                req.done = self.now()
                if req.make is not None:
                    req.phi0 = None  # rebuilt on demand; keeps host memory flat
                self.finished.append(req)

    def cancel(self, rid: int) -> bool:
        """Withdraws a queued or resident request: it finishes with the error
        "cancelled", and a resident one frees its slot and nodes at once (the
        other lattices are not touched).  Returns False if rid is not pending."""
        for r in self.queue:
            if r.rid == rid:
                self.queue.remove(r)
                break
        else:
            r = next((q for q in self.active.values() if q.rid == rid), None)
            if r is None:
                return False
            self.batch.remove(r.slot)
            del self.active[r.slot]
        r.error = "cancelled"
        r.done = self.now()
        self.finished.append(r)
        return True

    def run(self, arrivals: list[Request], max_wall_s: float = 1e9,
            on_tick: Callable[["Server"], None] | None = None) -> dict:
        """Replays an arrival trace in real time (request.arrival in seconds from
        start) until every request is finished.  on_tick(server) runs after every
        tick (e.g. to cancel requests)."""
        pending = collections.deque(sorted(arrivals, key=lambda r: r.arrival))
        self.t0 = self.clock()
        total_updates = 0
        while pending or self.queue or self.active:
            now = self.now()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            self._admit()
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(0.002, pending[0].arrival - self.now())))
                    continue
                if self.queue:  # nothing fits and nothing runs: cannot progress
                    for r in self.queue:
                        r.error = "cannot be admitted"
                        r.done = self.now()
                        self.finished.append(r)
                    self.queue.clear()
                break
            n = min([self.tick] + [req.steps - self.batch.t(s) for s, req in self.active.items()])
            n = max(1, n)
            total_updates += n * self.used_nodes()
            self.batch.step(n, use_graph=True)
            self._retire()
            if on_tick is not None:
                on_tick(self)
            if self.now() > max_wall_s:
                break
        wall = self.now()
        lat = np.array([r.latency for r in self.finished if r.error is None and r.latency is not None])
        return {
            "requests": len(self.finished),
            "failed": sum(1 for r in self.finished if r.error is not None),
            "wall_s": wall,
            "node_updates": total_updates,
            "MLUPS": total_updates / wall / 1e6 if wall > 0 else 0.0,
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        }

    def close(self) -> None:
        self.batch.close()
