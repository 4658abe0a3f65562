"""Host logic of the request loop: batch formation and HBM admission.

Uses stand-in plans (no GPU): each reports its resident bytes and a workspace
size linear in nrhs, which is all the admission rule reads.
"""
from __future__ import annotations

import collections

import pytest

from paper_1311_4257_amd import dfmm
from paper_1311_4257_amd.serve import Request, Server


class _Info:
    def __init__(self, b):
        self.device_bytes = b


class _FakePlan:
    def __init__(self, resident, per_rhs):
        self.resident, self.per_rhs = resident, per_rhs

    def info(self):
        return _Info(self.resident)

    def workspace_bytes(self, nrhs):
        return self.per_rhs * nrhs


class _F:
    def __init__(self, nrhs):
        self.shape = (nrhs, 10)


def _req(rid, plan, nrhs, t=0.0):
    return Request(rid, plan, _F(nrhs), None, t)


def test_batch_takes_queued_requests_in_order_up_to_the_rhs_cap():
    s = Server([_FakePlan(100, 1)], budget_bytes=10 ** 9, max_batch_rhs=16)
    q = collections.deque([_req(0, 0, 4), _req(1, 0, 4), _req(2, 0, 16), _req(3, 0, 1)])
    take, n = s._take(0, q)
    assert [r.rid for r in take] == [0, 1] and n == 8
    take, n = s._take(0, q)  # a request larger than the rest of the cap starts its own batch
    assert [r.rid for r in take] == [2] and n == 16
    take, n = s._take(0, q)
    assert [r.rid for r in take] == [3] and n == 1 and not q


def test_a_single_request_above_the_rhs_cap_still_runs_alone():
    s = Server([_FakePlan(0, 1)], budget_bytes=10 ** 9, max_batch_rhs=4)
    q = collections.deque([_req(0, 0, 16), _req(1, 0, 1)])
    take, n = s._take(0, q)
    assert [r.rid for r in take] == [0] and n == 16


def test_batch_request_count_is_capped():
    s = Server([_FakePlan(0, 1)], budget_bytes=10 ** 9, max_batch_rhs=10 ** 6)
    q = collections.deque([_req(i, 0, 1) for i in range(dfmm.MAX_BATCH + 5)])
    take, n = s._take(0, q)
    assert len(take) == dfmm.MAX_BATCH and n == dfmm.MAX_BATCH and len(q) == 5


def test_admission_keeps_the_footprint_within_the_budget():
    # resident 1000 + 1000; plan 0 costs 10 B per rhs, plan 1 already holds 8 rhs (80 B)
    plans = [_FakePlan(1000, 10), _FakePlan(1000, 10)]
    s = Server(plans, budget_bytes=2000 + 80 + 100, max_batch_rhs=64)
    s.cap[1] = 8
    assert s.footprint() == 2080
    q = collections.deque([_req(0, 0, 4), _req(1, 0, 4), _req(2, 0, 4)])
    take, n = s._take(0, q)  # 8 rhs -> 2160 fits, 12 rhs -> 2200 does not
    assert [r.rid for r in take] == [0, 1] and n == 8
    assert s.footprint(0, n) <= s.budget
    # the workspace is grow-only: once plan 0 holds 8 rhs, a batch of 8 costs nothing new
    s.cap[0] = 8
    take, n = s._take(0, q)
    assert [r.rid for r in take] == [2]


def test_a_request_that_never_fits_is_reported():
    s = Server([_FakePlan(1000, 10)], budget_bytes=1005, max_batch_rhs=64)
    q = collections.deque([_req(0, 0, 1)])
    take, n = s._take(0, q)
    assert take == [] and len(q) == 1


def test_single_mode_takes_one_request_per_pass():
    s = Server([_FakePlan(0, 1)], budget_bytes=10 ** 9, max_batch_rhs=64, mode="single")
    q = collections.deque([_req(0, 0, 1), _req(1, 0, 1)])
    take, _ = s._take(0, q)
    assert len(take) == 1


def test_unknown_mode_is_rejected():
    with pytest.raises(ValueError):
        Server([], budget_bytes=0, mode="fifo")
