"""Serving harness over the library's request loop (``dfmm.Server``).

An iterative boundary-integral solver issues one matvec per iteration; a
serving process holds the plans of several geometries and receives such
matvec requests as they come.  The loop itself is native (``dfmm_server_*``):
one stream per plan (default priority), a worker thread that starts a plan's
next pass, as one ``dfmm_apply_batch``, when its previous pass has finished,
from the plan's requests queued so far (submission order, up to
``max_batch_rhs`` right-hand sides and ``dfmm.MAX_BATCH`` requests, within an
HBM budget with grow-only workspaces), and completion reported by a host
function behind each pass.  ``mode="single"`` is the plain single-request
form: one request per pass and one pass at a time, in submission order.

This module replays a list of requests against such a server at their
arrival times (the calling thread sleeps until each arrival and submits it)
and reads back every request's submission and completion time on the
server's clock, for throughput and latency figures.
"""
from __future__ import annotations

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
    arrival: float     # seconds after the run starts (when it is submitted)
    submitted: float = float("nan")  # seconds after the run starts, server clock
    done: float = float("nan")
    ticket: int = -1

    @property
    def nrhs(self) -> int:
        return int(self.f.shape[0])

    @property
    def latency(self) -> float:
        return self.done - self.submitted


class Server:
    """A native server over ``plans`` plus the replay harness.  The plans must
    not be applied elsewhere while a run is in progress."""

    def __init__(self, plans, budget_bytes: int, max_batch_rhs: int = 32, mode: str = "batched"):
        if mode not in ("batched", "single"):
            raise ValueError(mode)
        self.plans = list(plans)
        self.mode = mode
        self.srv = dfmm.Server(self.plans, budget_bytes, max_batch_rhs, single=mode == "single")
        self.batches = []  # (plan, requests, nrhs) of the last run's passes, in launch order

    def footprint(self) -> int:
        return self.srv.footprint()

    def warm(self, sizes):
        """One pass per plan and batch size (workspace growth, launch shapes,
        chunk tables) before the timed runs, as far as the budget allows."""
        import torch

        for p, plan in enumerate(self.plans):
            for n in sorted(set(sizes)):
                f = torch.zeros((n, plan.N), dtype=torch.complex64, device="cuda")
                u = torch.empty_like(f)
                torch.cuda.synchronize()
                try:
                    self.srv.wait(self.srv.submit(p, f, u))
                except dfmm.DfmmError as e:
                    if e.status != dfmm.ENOMEM:
                        raise
                    break

    def run(self, requests) -> float:
        """Submit ``requests`` at their arrival times, wait for all of them, fill
        each one's ``submitted`` and ``done``; returns the span from the first
        submission to the last completion, in seconds."""
        import torch

        reqs = sorted(requests, key=lambda r: r.arrival)
        torch.cuda.synchronize()  # every request's densities are in place
        before = len(self.srv.passes())
        t0 = self.srv.now()
        for r in reqs:
            d = t0 + r.arrival - self.srv.now()
            if d > 0:
                time.sleep(d)
            r.ticket = self.srv.submit(r.plan, r.f, r.u)
        self.srv.drain()
        for r in reqs:
            ts, td = self.srv.wait(r.ticket)
            r.submitted, r.done = ts - t0, td - t0
        self.batches = self.srv.passes()[before:]
        return max(r.done for r in reqs) - min(r.submitted for r in reqs) if reqs else 0.0

    def close(self) -> None:
        self.srv.close()


def latency_stats(requests) -> dict:
    lat = np.array([r.latency for r in requests])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}
