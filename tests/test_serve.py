"""Serving scheduler on a simulated executor (CPU): continuous batching,
arrival-order admission, HBM budget, plan eviction, rejection, sequential
baseline and the latency summary."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2603_24881_amd.serve import FOCK, GRAD, Request, Scheduler, poisson_trace, summarize


class FakeExecutor:
    """Virtual clock; a round's eval batch costs 1 ms plus 1 ms per task, then
    each new request's Poisson step 1 ms (2 ms with its second stage); a single
    request 3 ms; records everything the scheduler asks for."""

    def __init__(self, plan_bytes, req_bytes, budget=None):
        self.t = 0.0
        self.pb = plan_bytes
        self.rb = req_bytes
        self.loaded = set()
        self.log = []
        self.active = set()
        self.peak = 0
        self.sched = None

    def plan_bytes(self, key):
        return self.pb[key]

    def request_bytes(self, key, kind):
        return self.rb[key] * (2 if kind == GRAD else 1)

    def load(self, key):
        assert key not in self.loaded
        self.loaded.add(key)
        self.log.append(("load", key))

    def unload(self, key):
        assert key in self.loaded
        assert all(r.system != key for r in self.active), "evicted a plan in use"
        self.loaded.remove(key)
        self.log.append(("unload", key))

    def _check_budget(self):
        used = sum(self.pb[k] for k in self.loaded) + sum(self.request_bytes(r.system, r.kind) for r in self.active)
        self.peak = max(self.peak, used)
        assert used <= self.sched.budget

    def begin(self, r):
        assert r.system in self.loaded
        self.active.add(r)
        self._check_budget()
        self.log.append(("begin", r.rid))

    def round(self, s0, s1, finish_new=False):
        assert all(r.stage == 0 for r in s0) and all(r.stage == 1 for r in s1)
        self.log.append(("round", [r.rid for r in s0], [r.rid for r in s1], finish_new))
        self.t += 1e-3 * (1 + len(s0) + len(s1))        # the batch
        t_s1 = self.t if s1 else None
        self.t += 1e-3 * len(s0) * (2 if finish_new else 1)   # Poisson (+ second stage)
        return t_s1

    def single(self, r):
        self.log.append(("single", r.rid))
        self.t += 3e-3

    def end(self, r):
        self.active.discard(r)
        r.result = {"E_J": 1.0}

    def now(self):
        return self.t

    def sleep_until(self, t):
        assert t >= self.t - 1e-15
        self.t = t


def _sched(ex, budget, max_active=16):
    s = Scheduler(ex, budget, max_active=max_active)
    ex.sched = s
    return s


def test_every_request_completes_in_one_or_two_rounds():
    """Two rounds (first stage, then second stage), or one when nobody was
    waiting as its first round started."""
    ex = FakeExecutor({"a": 10, "b": 20}, {"a": 1, "b": 2})
    s = _sched(ex, 1000, max_active=3)
    reqs = [Request(i, FOCK if i % 2 else GRAD, "ab"[i % 2], 0.0005 * i) for i in range(20)]
    s.run(reqs)
    fused = 0
    for r in reqs:
        assert r.error is None and r.done >= r.admitted >= r.arrival
        rounds = [e for e in ex.log if e[0] == "round" and (r.rid in e[1] or r.rid in e[2])]
        assert r.rid in rounds[0][1]
        if rounds[0][3]:
            assert len(rounds) == 1
            fused += 1
        else:
            assert len(rounds) == 2 and r.rid in rounds[1][2]
    assert 0 < fused < len(reqs)


def test_lone_request_finishes_in_one_round():
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000)
    r = Request(0, FOCK, "a", 0.0)
    s.run([r])
    assert [e for e in ex.log if e[0] == "round"] == [("round", [0], [], True)]
    assert r.done == pytest.approx(0.004)


def test_waiting_requests_join_the_next_round():
    """Under load the new requests' first stage shares the launches of the
    previous ones' second stage."""
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000, max_active=2)
    reqs = [Request(i, FOCK if i % 2 else GRAD, "a", 0.0) for i in range(5)]
    s.run(reqs)
    rounds = [e for e in ex.log if e[0] == "round"]
    assert rounds == [("round", [0, 1], [], False), ("round", [2, 3], [0, 1], False),
                      ("round", [4], [2, 3], True)]


def test_second_stage_completes_with_the_batch():
    """A request in its second stage is complete when the round's batch is,
    not after the Poisson steps of the requests that joined the round."""
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000, max_active=2)
    reqs = [Request(i, FOCK, "a", 0.0) for i in range(3)]
    s.run(reqs)
    # first round: [0, 1] first stage (batch 3 ms + Poisson 2 ms) -> t = 5 ms
    # second round: [2] first stage, [0, 1] second (batch 4 ms -> 9 ms; Poisson and
    # the fused second stage of 2: 2 ms -> 11 ms)
    assert reqs[0].done == pytest.approx(0.009) and reqs[1].done == pytest.approx(0.009)
    assert reqs[2].done == pytest.approx(0.011)


def test_admission_in_arrival_order_under_budget():
    """A large head request waits for memory; smaller ones behind it do not overtake."""
    ex = FakeExecutor({"a": 10, "b": 10}, {"a": 5, "b": 30})
    s = _sched(ex, 100)
    reqs = [Request(0, GRAD, "b", 0.0), Request(1, GRAD, "b", 0.0001),
            Request(2, FOCK, "a", 0.0002), Request(3, FOCK, "a", 0.0003)]
    s.run(reqs)
    begins = [e[1] for e in ex.log if e[0] == "begin"]
    assert begins == [0, 1, 2, 3]
    assert reqs[1].admitted >= reqs[0].done        # two 60-byte gradient requests and the plan exceed 100
    assert ex.peak <= 100


def test_idle_plans_are_evicted_lru_and_busy_ones_kept():
    ex = FakeExecutor({"a": 40, "b": 40, "c": 40}, {"a": 1, "b": 1, "c": 1})
    s = _sched(ex, 90)
    reqs = [Request(0, FOCK, "a", 0.0), Request(1, FOCK, "b", 0.01), Request(2, FOCK, "c", 0.02),
            Request(3, FOCK, "a", 0.03)]
    s.run(reqs)
    assert all(r.error is None for r in reqs)
    ev = [e for e in ex.log if e[0] in ("load", "unload")]
    assert ev == [("load", "a"), ("load", "b"), ("unload", "a"), ("load", "c"), ("unload", "b"), ("load", "a")]


def test_request_that_never_fits_is_rejected():
    ex = FakeExecutor({"a": 10, "big": 500}, {"a": 1, "big": 1})
    s = _sched(ex, 100)
    reqs = [Request(0, FOCK, "a", 0.0), Request(1, FOCK, "big", 0.0), Request(2, GRAD, "a", 0.0)]
    s.run(reqs)
    assert reqs[1].error and math.isnan(reqs[1].done)
    assert reqs[0].error is None and reqs[2].error is None
    assert summarize(reqs)["rejected"] == 1 and summarize(reqs)["completed"] == 2


def test_max_active_is_respected():
    ex = FakeExecutor({"a": 1}, {"a": 1})
    s = _sched(ex, 10 ** 6, max_active=3)
    reqs = [Request(i, FOCK, "a", 0.0) for i in range(10)]
    s.run(reqs)
    for e in ex.log:
        if e[0] == "round":
            assert len(e[1]) <= 3 and len(e[2]) <= 3


def test_sequential_baseline_and_summary():
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000)
    reqs = [Request(i, FOCK, "a", 0.001 * i) for i in range(5)]
    s.run_sequential(reqs)
    lat = [r.latency for r in reqs]
    # 3 ms each, arrivals 1 ms apart: request i waits 2 ms per earlier request
    np.testing.assert_allclose(lat, [0.003 * (i + 1) - 0.001 * i for i in range(5)], atol=1e-12)
    sm = summarize(reqs)
    assert sm["completed"] == 5
    assert sm["p50_ms"] == pytest.approx(np.percentile(np.array(lat) * 1e3, 50))
    assert sm["p99_ms"] == pytest.approx(np.percentile(np.array(lat) * 1e3, 99))
    assert sm["req_per_s"] == pytest.approx(5 / (reqs[-1].done - reqs[0].arrival))


def test_poisson_trace_statistics():
    tr = poisson_trace(4000, 20.0, seed=2000)
    gaps = np.diff([r.arrival for r in tr])
    assert tr[0].arrival == 0.0 and np.all(gaps >= 0)
    assert abs(gaps.mean() - 0.05) < 0.005
    kinds = np.array([r.kind == GRAD for r in tr])
    assert abs(kinds.mean() - 0.5) < 0.03
    sizes = {r.system.split("g")[0] for r in tr}
    assert sizes == {"w8", "w16", "w32", "w64", "w128", "w256"}
    assert poisson_trace(50, 20.0)[7].arrival == poisson_trace(50, 20.0)[7].arrival
