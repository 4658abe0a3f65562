"""Continuous-batching request loop over plans resident on one GPU.

An iterative boundary-integral solver issues one matvec per iteration; a
serving process holds the plans of several geometries (each plan keeps its
tree, lists and translation operators on the device) and receives such
matvec requests as they come.  This loop:

* keeps one stream per plan (default priority) and at most one batch in flight
  per plan; batches of different plans run concurrently on the device;
* forms a plan's next batch, when its previous one has finished, from the
  requests of that plan queued so far, in arrival order, up to ``max_batch_rhs``
  right-hand sides and ``dfmm.MAX_BATCH`` requests, and only while the HBM
  footprint stays within ``budget_bytes``: the resident plans plus every plan's
  workspace at the largest batch it has run (the workspace is grow-only);
* runs a batch as one ``dfmm_apply_batch`` pass (densities gathered from the
  requests' own buffers, potentials scattered to theirs), so requests that
  arrive while others are on the GPU join the next pass of their plan.

``mode="single"`` is the plain single-request form for comparison: one request
per pass and one pass in flight at a time, in arrival order.

Completion times come from timing events recorded after each pass on the
plan's stream, read against an event recorded when the run starts, so a
latency is (pass end on the GPU) - (arrival on the host clock) without host
polling granularity.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import dfmm


@dataclasses.dataclass
class Request:
    rid: int
    plan: int          # index into the server's plans
    f: object          # (nrhs, N) complex64 device tensor
    u: object          # (nrhs, N) complex64 device tensor, written by the pass
    arrival: float     # seconds after the run starts
    done: float = float("nan")

    @property
    def nrhs(self) -> int:
        return int(self.f.shape[0])


class Server:
    def __init__(self, plans, budget_bytes: int, max_batch_rhs: int = 32, mode: str = "batched", device=0):
        if mode not in ("batched", "single"):
            raise ValueError(mode)
        self.plans = list(plans)
        self.budget = int(budget_bytes)
        self.max_rhs = int(max_batch_rhs)
        self.mode = mode
        self.device = device
        self.streams = None  # created on first use (one per plan)
        self.resident = sum(int(p.info().device_bytes) for p in self.plans)
        self.cap = [0] * len(self.plans)  # largest batch nrhs run per plan (workspace size)
        self._wsb = {}
        self.batches = []  # (plan, [rid...], nrhs) of the last run, in launch order

    def ws_bytes(self, p: int, nrhs: int) -> int:
        if nrhs <= 0:
            return 0
        key = (p, nrhs)
        if key not in self._wsb:
            self._wsb[key] = self.plans[p].workspace_bytes(nrhs)
        return self._wsb[key]

    def footprint(self, p: int | None = None, nrhs: int = 0) -> int:
        """HBM bytes held with plan p's workspace grown to nrhs (current state if p is None)."""
        tot = self.resident
        for q in range(len(self.plans)):
            c = self.cap[q]
            if q == p:
                c = max(c, nrhs)
            tot += self.ws_bytes(q, c)
        return tot

    def _dev(self):
        import torch

        if self.streams is None:
            self.device = torch.device("cuda", self.device) if isinstance(self.device, int) else self.device
            self.streams = [torch.cuda.Stream(device=self.device) for _ in self.plans]
        return self.device

    def warm(self, sizes):
        """Run one pass per plan and batch size (workspace growth, tuning, chunk
        tables) before the timed runs, as far as the budget allows."""
        import torch

        self._dev()
        for p, plan in enumerate(self.plans):
            for n in sorted(set(sizes)):
                if self.footprint(p, n) > self.budget:
                    break
                f = torch.zeros((n, plan.N), dtype=torch.complex64, device=self.device)
                u = torch.empty_like(f)
                plan.apply_batch([f], [u], self.streams[p])
                self.cap[p] = max(self.cap[p], n)
            self.streams[p].synchronize()

    def _take(self, p: int, q: collections.deque):
        """Requests of plan p's next batch (removed from q), or [] if none fits."""
        take, n = [], 0
        while q and len(take) < dfmm.MAX_BATCH:
            r = q[0]
            if take and (n + r.nrhs > self.max_rhs or self.mode == "single"):
                break
            if self.footprint(p, n + r.nrhs) > self.budget:
                break
            take.append(q.popleft())
            n += r.nrhs
        return take, n

    def run(self, requests):
        """Serve ``requests`` (sorted by arrival); fills each one's ``done`` and
        returns the run's makespan in seconds."""
        import torch

        self._dev()
        reqs = sorted(requests, key=lambda r: r.arrival)
        P = len(self.plans)
        queues = [collections.deque() for _ in range(P)]
        fifo = collections.deque()  # single mode: one queue over all plans
        inflight = [None] * P       # (event, requests)
        ends = []                   # (event, requests) of every pass
        self.batches = []
        torch.cuda.synchronize(self.device)
        start = torch.cuda.Event(enable_timing=True)
        start.record(torch.cuda.current_stream(self.device))
        t0 = time.perf_counter()
        i, busy = 0, 0
        while i < len(reqs) or busy or any(queues) or fifo:
            now = time.perf_counter() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                r = reqs[i]
                (fifo if self.mode == "single" else queues[r.plan]).append(r)
                i += 1
            for p in range(P):
                if inflight[p] is not None and inflight[p][0].query():
                    inflight[p] = None
                    busy -= 1
            if self.mode == "single":
                if busy == 0 and fifo:
                    r = fifo[0]
                    self._launch(r.plan, [fifo.popleft()], r.nrhs, inflight, ends)
                    busy += 1
                continue
            # idle plans, oldest queued request first
            idle = [p for p in range(P) if inflight[p] is None and queues[p]]
            for p in sorted(idle, key=lambda p: queues[p][0].arrival):
                take, n = self._take(p, queues[p])
                if take:
                    self._launch(p, take, n, inflight, ends)
                    busy += 1
            if busy == 0 and any(queues):
                raise RuntimeError("a request does not fit the HBM budget even alone")
        torch.cuda.synchronize(self.device)
        last = 0.0
        for ev, batch in ends:
            t = start.elapsed_time(ev) * 1e-3
            for r in batch:
                r.done = t
            last = max(last, t)
        first = reqs[0].arrival if reqs else 0.0
        return last - first

    def _launch(self, p, batch, n, inflight, ends):
        import torch

        s = self.streams[p]
        self.plans[p].apply_batch([r.f for r in batch], [r.u for r in batch], s)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(s)
        self.cap[p] = max(self.cap[p], n)
        inflight[p] = (ev, batch)
        ends.append((ev, batch))
        self.batches.append((p, [r.rid for r in batch], n))


def latency_stats(requests) -> dict:
    lat = np.array([r.done - r.arrival for r in requests])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}
