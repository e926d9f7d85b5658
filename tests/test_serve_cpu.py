"""Host-side tests of the continuous-batching server with an oracle-backed fake executor.

The fake executor keeps the same slot/step interface as the GPU executor: it counts pipeline
steps and, when a request finishes, computes its result with the FP64 oracle.  This checks
admission by footprint and slots, backfill, cancellation, failure isolation and bookkeeping
without a GPU.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import Problem, ridc_pipelined
from paper_1209_4297_amd.serve import Request, Server


class FakeExecutor:
    def __init__(self, bytes_per_unknown=136):
        self.bpu = bytes_per_unknown
        self.slots = {}
        self.next = 0
        self.log = []

    def footprint(self, req):
        if req.prob["n"] < 2:
            return 0
        return req.unknowns * self.bpu

    def start(self, req):
        if req.prob.get("fail_start"):
            raise RuntimeError("device allocation failed")
        P = req.prob["order"]
        steps = req.nsteps + P * (P - 1) // 2 if req.nsteps > 0 else 0
        slot = self.next
        self.next += 1
        self.slots[slot] = [req, steps]
        self.log.append(("start", req.rid))
        return slot

    def advance(self, slots, k):
        self.log.append(("advance", tuple(sorted(self.slots[s][0].rid for s in slots)), k))
        for s in slots:
            self.slots[s][1] = max(0, self.slots[s][1] - k)

    def remaining(self, slot):
        return self.slots[slot][1]

    def finish(self, slot):
        req = self.slots[slot][0]
        out = ridc_pipelined(Problem.from_dict(req.prob), np.asarray(req.u0), req.nsteps,
                             req.prob["order"])[-1]
        if not np.all(np.isfinite(out)):
            raise FloatingPointError("result holds a NaN or Inf")
        return out

    def release(self, slot):
        self.slots.pop(slot)
        self.log.append(("release", slot))


def _req(rid, n=16, order=3, nt=10, t=0.0, **extra):
    prob, u0 = workloads.config_reacdiff_1d(n=n, nt=nt, order=order, T=nt * 1e-3)
    prob.update(extra)
    return Request(rid=rid, prob=prob, u0=u0, nsteps=nt, prec="fp64", t_arrival=t)


def test_admission_respects_budget_and_slots():
    ex = FakeExecutor()
    budget = 3 * 16 * 136                       # room for three n=16 requests
    srv = Server(ex, hbm_budget=budget, max_slots=2, tick_steps=4)
    for i in range(5):
        srv.submit(_req(i))
    srv.tick()
    assert len(srv.running) == 2 and len(srv.queue) == 3      # slot-limited
    while not srv.idle():
        srv.tick()
        assert srv.used <= budget and len(srv.running) <= 2
    assert sorted(r.rid for r in srv.done) == list(range(5))
    assert all(r.status == "done" for r in srv.done)
    assert srv.peak_used <= budget


def test_results_match_oracle_alone():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10**9, max_slots=8, tick_steps=3)
    reqs = [_req(i, n=8 + 4 * i, order=2 + i % 3, nt=6 + i) for i in range(6)]
    for r in reqs:
        srv.submit(r)
    while not srv.idle():
        srv.tick()
    for r in reqs:
        alone = ridc_pipelined(Problem.from_dict(r.prob), r.u0, r.nsteps, r.prob["order"])[-1]
        np.testing.assert_array_equal(r.result, alone)


def test_late_arrivals_join_running_batch():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10**9, max_slots=8, tick_steps=2)
    srv.submit(_req(0, nt=20))
    srv.tick()
    srv.submit(_req(1, nt=4))                   # arrives while request 0 is mid-flight
    srv.tick()
    adv = [e for e in ex.log if e[0] == "advance"]
    assert adv[0][1] == (0,) and adv[1][1] == (0, 1)      # same grouped advance
    while not srv.idle():
        srv.tick()
    order = [r.rid for r in srv.done]
    assert order == [1, 0]                      # the short late request finishes first


def test_backfill_lets_small_requests_pass_a_large_one():
    ex = FakeExecutor()
    budget = 100 * 136
    srv = Server(ex, hbm_budget=budget, max_slots=8, tick_steps=4)
    srv.submit(_req(0, n=64, nt=30))            # 64 unknowns resident
    srv.tick()
    srv.submit(_req(1, n=64, nt=5))             # does not fit next to request 0
    srv.submit(_req(2, n=16, nt=5))             # fits
    srv.tick()
    assert {srv.running[s][0].rid for s in srv.running} == {0, 2}
    while not srv.idle():
        srv.tick()
    assert all(r.status == "done" for r in srv.done)


def test_rejects_oversized_and_invalid():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10 * 136, max_slots=4)
    srv.submit(_req(0, n=64))
    bad = _req(1)
    bad.prob["n"] = 1
    srv.submit(bad)
    assert [r.status for r in srv.done] == ["rejected", "rejected"]
    assert srv.idle()


def test_cancel_queued_and_running():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10**9, max_slots=1, tick_steps=1)
    srv.submit(_req(0, nt=50))
    srv.submit(_req(1, nt=5))
    srv.tick()
    assert srv.cancel(1)                        # still queued
    assert srv.cancel(0)                        # running: its slot is released
    assert not srv.cancel(7)
    assert srv.idle() and srv.used == 0
    assert {r.rid: r.status for r in srv.done} == {1: "cancelled", 0: "cancelled"}
    assert ("release", 0) in ex.log


def test_failures_are_isolated():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10**9, max_slots=8, tick_steps=5)
    nan = _req(0, nt=8)
    nan.u0 = nan.u0.copy()
    nan.u0[3] = math.nan
    srv.submit(nan)
    srv.submit(_req(1, nt=8, fail_start=True))
    srv.submit(_req(2, nt=8))
    while not srv.idle():
        srv.tick()
    st = {r.rid: r.status for r in srv.done}
    assert st == {0: "failed", 1: "failed", 2: "done"}
    assert srv.used == 0


def test_run_reports_latency_percentiles():
    ex = FakeExecutor()
    t = [0.0]

    def clock():
        t[0] += 1e-3
        return t[0]

    srv = Server(ex, hbm_budget=10**9, max_slots=4, tick_steps=4, clock=clock)
    arrivals = [_req(i, nt=6, t=0.002 * i) for i in range(10)]
    stats = srv.run(arrivals)
    assert stats["completed"] == 10
    assert stats["p50_latency_s"] > 0 and stats["p99_latency_s"] >= stats["p50_latency_s"]
    assert stats["completed_grid_point_steps_per_s"] > 0
