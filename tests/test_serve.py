"""Serving scheduler on a simulated executor (CPU): continuous batching on
lanes, admission while rounds run, arrival-order admission, HBM budget, plan
eviction, rejection, the active-request cap, the sequential baseline and the
latency summary."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2603_24881_amd.serve import FOCK, GRAD, Request, Scheduler, poisson_trace, summarize


class FakeExecutor:
    """Virtual clock.  A round on a lane costs 1 ms plus each request's cost
    (``cost[system]``, 1 ms by default); lanes run independently; a single
    request costs 1 ms plus its cost.  Records everything the scheduler asks
    for and checks the budget and the active-request cap."""

    def __init__(self, plan_bytes, req_bytes, cost=None, lanes=2, limits=None):
        self.t = 0.0
        self.pb = plan_bytes
        self.rb = req_bytes
        self.cost_of = cost or {}
        self.n_lanes = lanes
        self.limits = limits or {}
        self.loaded = set()
        self.log = []
        self.active = set()
        self.peak = 0
        self.peak_active = 0
        self.lane_busy = {}
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
        self.peak_active = max(self.peak_active, len(self.active))
        assert len(self.active) <= self.sched.max_active
        self._check_budget()
        self.log.append(("begin", r.rid, self.t))

    def _cost(self, r):
        return self.cost_of.get(r.system, 1e-3)

    def cost(self, key):      # the scheduler's work estimate
        return self.cost_of.get(key, 1e-3)

    def lane_limit(self, lane):
        return self.limits.get(lane)

    def launch(self, batch, lane):
        assert 0 <= lane < self.n_lanes
        assert self.lane_busy.get(lane, -1.0) <= self.t, "launched on a busy lane"
        fin = self.t + 1e-3 + sum(self._cost(r) for r in batch)
        self.lane_busy[lane] = fin
        self.log.append(("launch", lane, [r.rid for r in batch], self.t))
        return fin

    def done(self, h):
        return self.t >= h

    def wait(self, t_next, handles):
        cands = list(handles) + ([t_next] if t_next is not None else [])
        assert cands, "wait with nothing to wait for"
        t = min(cands)
        assert t >= self.t - 1e-15
        self.t = max(self.t, t)

    def single(self, r):
        self.log.append(("single", r.rid))
        self.t += 1e-3 + self._cost(r)

    def end(self, r):
        self.active.discard(r)
        r.result = {"E_J": 1.0}

    def now(self):
        return self.t

    def sleep_until(self, t):
        assert t >= self.t - 1e-15
        self.t = t


def _sched(ex, budget, max_active=32, max_batch=16):
    s = Scheduler(ex, budget, max_active=max_active, max_batch=max_batch)
    ex.sched = s
    return s


def _launches(ex):
    return [e for e in ex.log if e[0] == "launch"]


def test_every_request_runs_in_exactly_one_round():
    ex = FakeExecutor({"a": 10, "b": 20}, {"a": 1, "b": 2})
    s = _sched(ex, 1000, max_active=3)
    reqs = [Request(i, FOCK if i % 2 else GRAD, "ab"[i % 2], 0.0005 * i) for i in range(20)]
    s.run(reqs)
    for r in reqs:
        assert r.error is None and r.done >= r.admitted >= r.arrival
        rounds = [e for e in _launches(ex) if r.rid in e[2]]
        assert len(rounds) == 1
        assert r.done >= rounds[0][3] + 1e-3
    assert sum(s.rounds) == len(reqs) and max(s.rounds) > 1


class TickingExecutor(FakeExecutor):
    """A host clock that moves on by itself: every reading is 0.3 ms later."""

    def now(self):
        self.t += 3e-4
        return self.t


@pytest.mark.parametrize("gap_ms", [2.75, 2.95, 3.05, 3.15, 3.35])
def test_arrival_between_clock_readings_of_an_idle_server(gap_ms):
    """A request that arrives after the server, idle again once a 2 ms round
    ends, has read the clock for admission but before it reads it again to
    decide whether to wait, is admitted on the next trip (no accounting
    error).  With clock readings 0.3 ms apart, the gaps of 2.95 to 3.15 ms put
    the arrival of the second request between the two readings."""
    ex = TickingExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000)
    reqs = [Request(0, FOCK, "a", 0.0), Request(1, FOCK, "a", gap_ms * 1e-3)]
    s.run(reqs)
    assert all(r.error is None and r.done >= r.admitted >= r.arrival for r in reqs)
    assert s.rounds == [1, 1]


def test_lone_request_is_one_round_on_a_free_lane():
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000)
    r = Request(0, FOCK, "a", 0.0)
    s.run([r])
    assert [e[2] for e in _launches(ex)] == [[0]]
    assert r.done == pytest.approx(0.002)


def test_arrivals_are_admitted_while_a_round_runs_and_batched_next():
    """One lane: requests that arrive while a round is on the device are
    admitted at once and share the next round."""
    ex = FakeExecutor({"a": 10}, {"a": 1}, lanes=1)
    s = _sched(ex, 1000)
    arr = [0.0, 0.0005, 0.0005, 0.001]
    reqs = [Request(i, FOCK, "a", t) for i, t in enumerate(arr)]
    s.run(reqs)
    assert [e[2] for e in _launches(ex)] == [[0], [1, 2, 3]]
    for r in reqs:
        assert r.admitted == pytest.approx(r.arrival)      # not held back by the running round
    assert reqs[0].done == pytest.approx(0.002)
    # second round: starts when the first ends (2 ms), 1 ms + 3 x 1 ms
    assert all(r.done == pytest.approx(0.006) for r in reqs[1:])


def test_a_small_request_does_not_wait_behind_a_large_one():
    """Two lanes: a small request arriving while a large one runs takes the
    free lane and finishes first."""
    ex = FakeExecutor({"big": 10, "small": 10}, {"big": 1, "small": 1}, cost={"big": 0.02, "small": 0.001})
    s = _sched(ex, 1000)
    reqs = [Request(0, FOCK, "big", 0.0), Request(1, FOCK, "small", 0.0005)]
    s.run(reqs)
    la = _launches(ex)
    assert [e[1] for e in la] == [0, 1] and la[1][3] == pytest.approx(0.0005)
    assert reqs[1].done == pytest.approx(0.0025) and reqs[0].done == pytest.approx(0.021)


def test_waiting_requests_are_split_between_free_lanes():
    ex = FakeExecutor({"a": 10}, {"a": 1})
    s = _sched(ex, 1000)
    reqs = [Request(i, FOCK, "a", 0.0) for i in range(6)]
    s.run(reqs)
    assert [(e[1], e[2]) for e in _launches(ex)] == [(0, [0, 1, 2]), (1, [3, 4, 5])]


def test_heavy_requests_take_lane_zero_one_round_at_a_time():
    """Lane 1 takes light requests only: two heavy requests run one after the
    other on lane 0 while the light ones pass beside them on lane 1."""
    ex = FakeExecutor({"big": 10, "small": 10}, {"big": 1, "small": 1}, cost={"big": 0.02, "small": 0.001},
                      limits={1: 0.005})
    s = _sched(ex, 1000, max_batch=1)
    reqs = [Request(0, FOCK, "big", 0.0), Request(1, FOCK, "big", 0.0), Request(2, FOCK, "small", 0.0),
            Request(3, FOCK, "small", 0.001)]
    s.run(reqs)
    lanes = {e[2][0]: e[1] for e in _launches(ex)}
    assert lanes == {0: 0, 1: 0, 2: 1, 3: 1}
    assert reqs[0].done == pytest.approx(0.021) and reqs[1].done == pytest.approx(0.042)
    assert reqs[2].done == pytest.approx(0.002) and reqs[3].done == pytest.approx(0.004)


def test_rounds_group_requests_of_similar_work():
    """A small request does not join the round of a large one: rounds hold
    requests within group_ratio of the oldest waiting one's estimate."""
    ex = FakeExecutor({"big": 10, "mid": 10, "small": 10}, {"big": 1, "mid": 1, "small": 1},
                      cost={"big": 0.02, "mid": 0.012, "small": 0.001}, lanes=1)
    s = _sched(ex, 1000)
    reqs = [Request(0, FOCK, "small", 0.0), Request(1, FOCK, "big", 0.0005), Request(2, FOCK, "small", 0.0006),
            Request(3, FOCK, "mid", 0.0007), Request(4, FOCK, "small", 0.0008)]
    s.run(reqs)
    assert [e[2] for e in _launches(ex)] == [[0], [1, 3], [2, 4]]


def test_batches_are_capped():
    ex = FakeExecutor({"a": 10}, {"a": 1}, lanes=1)
    s = _sched(ex, 1000, max_batch=4)
    reqs = [Request(i, FOCK, "a", 0.0) for i in range(10)]
    s.run(reqs)
    assert s.rounds == [4, 4, 2]


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
    assert ex.peak_active == 3 and all(r.error is None for r in reqs)


def test_sequential_baseline_and_summary():
    ex = FakeExecutor({"a": 10}, {"a": 1}, cost={"a": 0.002})
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


def test_continuous_beats_sequential_on_a_mixed_trace():
    """Large and small requests at a moderate rate (the simulated lanes do
    not slow each other down, so this checks the scheduling, not the device):
    small requests stop queueing behind large ones and p99 drops."""
    sizes = {"w8g0": 0.001, "w256g0": 0.02}
    rng = np.random.default_rng(3)
    arr = np.cumsum(rng.exponential(1 / 60.0, size=300))
    keys = rng.choice(list(sizes), size=300)

    def trace():
        return [Request(i, FOCK, str(keys[i]), float(arr[i])) for i in range(300)]

    def executor():
        return FakeExecutor({k: 1 for k in sizes}, {k: 1 for k in sizes}, cost=sizes)

    cont, seq = trace(), trace()
    _sched(executor(), 10 ** 6).run(cont)
    _sched(executor(), 10 ** 6).run_sequential(seq)
    assert summarize(cont)["p99_ms"] < summarize(seq)["p99_ms"]


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


def _heavy_light_run(heavy_alone):
    ex = FakeExecutor({"h": 10, "l": 1}, {"h": 1, "l": 1}, cost={"h": 5e-3, "l": 1e-4}, lanes=2, limits={1: 1e-3})
    s = Scheduler(ex, 1000, heavy_alone=heavy_alone)
    ex.sched = s
    reqs = [Request(i, FOCK, "h", 0.0) for i in range(3)] + [Request(3 + i, FOCK, "l", 0.0) for i in range(4)]
    s.run(reqs)
    assert all(r.error is None for r in reqs)
    heavy = [e for e in _launches(ex) if any(reqs[q].system == "h" for q in e[2])]
    light = [e for e in _launches(ex) if all(reqs[q].system == "l" for q in e[2])]
    return heavy, light, reqs


def test_heavy_requests_run_in_rounds_of_their_own():
    """A request too heavy for the restricted lane is not batched with
    another (it would only wait for it); light requests still share rounds."""
    heavy, light, reqs = _heavy_light_run(True)
    assert len(heavy) == 3 and all(len(e[2]) == 1 for e in heavy)
    assert max(len(e[2]) for e in light) > 1
    first = min(reqs[:3], key=lambda r: r.done)
    heavy2, _, reqs2 = _heavy_light_run(False)
    assert any(len(e[2]) > 1 for e in heavy2)
    assert first.done < min(r.done for r in reqs2[:3])   # the first heavy request completes sooner
