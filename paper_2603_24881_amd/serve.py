"""Serving: continuous batching of Fock-build and gradient requests.

A request names a resident system (its plan stays on the device between
requests) and carries a density matrix D.  A Fock request returns the
Coulomb matrix J = eval_mat(v_H) and E_J; a gradient request returns
dE_J/dR = eval_grad(D, v_H) and E_J, where v_H is the Hartree potential of
rho = eval_rho(D) from the multigrid Poisson step.

The server keeps a few lanes, each a device stream.  Whenever a lane is free
and admitted requests are waiting, the lane takes a batch of them and runs
their whole request as one round: one ``gpw_eval_batch`` call with the
collocation of every request in the batch (requests of different systems and
sizes share the same launches), the Poisson step of each, one
``gpw_eval_batch`` call with the integration or gradient of each, and an
event at the end.  Rounds on different lanes run on the device at the same
time, so a small request does not wait behind a large one while a lane is
free.  The host loop never blocks on the device: it polls the lanes' events,
hands results back as soon as their round has completed (that is the time
a request is stamped done), admits arrivals while rounds run, and otherwise
sleeps until the next arrival or completion.  Admission is in arrival order,
while the number of admitted, unfinished requests stays within
``max_active`` and their device memory (plus that of their plan, when it is
not resident) fits the HBM budget; idle plans are evicted least recently
used first to make room.  A request that can never fit is rejected.  With
several free lanes the waiting requests are split between them; a batch
holds at most ``max_batch`` requests, of work estimates within
``group_ratio`` of the oldest waiting request's (a small request then does
not wait for a large one that shares its round).

``run_sequential`` is the baseline: the same requests, one at a time in
arrival order, with the plain single calls, each stamped done after the
device has finished it.

The scheduler talks to an executor (``GPUExecutor`` here; tests use a
simulated one) through: n_lanes, cost, plan_bytes, request_bytes, load,
unload, begin, launch, done, wait, single, end, now, sleep_until.
"""
from __future__ import annotations

import math
import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

FOCK, GRAD = "fock", "grad"


@dataclass(eq=False)
class Request:
    rid: int
    kind: str                 # FOCK or GRAD
    system: str               # key of a registered system
    arrival: float            # seconds after the start of the run
    seed: int = 0             # seed of the request's density matrix
    admitted: float = math.nan
    done: float = math.nan
    stage: int = 0            # 0: collocation pending, 1: integration pending
    error: str | None = None
    result: dict | None = None
    state: dict = field(default_factory=dict)   # executor-owned buffers

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_trace(n, rate, sizes=(8, 16, 32, 64, 128, 256), geometries=2, grad_fraction=0.5, seed=2000):
    """n requests with exponential inter-arrival times of mean 1/rate; system
    size uniform over ``sizes``, geometry uniform over ``geometries``, kind
    GRAD with probability grad_fraction."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    size = rng.choice(np.asarray(sizes), size=n)
    geo = rng.integers(0, geometries, size=n)
    kind = rng.random(n) < grad_fraction
    return [Request(i, GRAD if kind[i] else FOCK, system_key(int(size[i]), int(geo[i])), float(t[i]),
                    seed=int(rng.integers(1 << 30))) for i in range(n)]


def system_key(n_waters, geometry):
    return f"w{n_waters}g{geometry}"


class Scheduler:
    def __init__(self, executor, budget_bytes, max_active=32, max_batch=16, group_ratio=2.0, heavy_alone=True):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.max_batch = int(max_batch)
        self.group_ratio = group_ratio
        # heavy_alone: a request too heavy for every restricted lane runs in a
        # round of its own (batching gains it nothing: its kernels fill the
        # device; a second heavy request in its round only delays it)
        self.heavy_alone = bool(heavy_alone)
        self.lanes = int(executor.n_lanes)
        self.used = 0
        self.n_active = 0                 # admitted, not yet done
        self.resident = OrderedDict()     # key -> plan bytes, least recently used first
        self.users = {}                   # key -> active requests on that plan
        self.rounds = []                  # per launched round: number of requests

    # ---------------------------------------------------------- memory
    def _need(self, r):
        need = self.ex.request_bytes(r.system, r.kind)
        if r.system not in self.resident:
            need += self.ex.plan_bytes(r.system)
        return need

    def _fits_ever(self, r):
        return self.ex.request_bytes(r.system, r.kind) + self.ex.plan_bytes(r.system) <= self.budget

    def _reserve(self, r):
        """Reserve memory for r (loading its plan); False if it does not fit now."""
        need = self._need(r)
        if self.used + need > self.budget:
            for key in list(self.resident):
                if self.used + need <= self.budget:
                    break
                if key != r.system and self.users.get(key, 0) == 0:
                    self.ex.unload(key)
                    self.used -= self.resident.pop(key)
        if self.used + need > self.budget:
            return False
        if r.system not in self.resident:
            self.ex.load(r.system)
            self.resident[r.system] = self.ex.plan_bytes(r.system)
        self.resident.move_to_end(r.system)
        self.used += need
        self.users[r.system] = self.users.get(r.system, 0) + 1
        return True

    def _release(self, r):
        self.used -= self.ex.request_bytes(r.system, r.kind)
        self.users[r.system] -= 1
        self.n_active -= 1

    def _admit(self, pending, queue, now):
        """Admit the arrived requests in arrival order while slots and memory allow."""
        while pending and pending[0].arrival <= now and self.n_active < self.max_active:
            r = pending[0]
            if not self._fits_ever(r):
                pending.popleft()
                r.error = "request and plan exceed the HBM budget"
                continue
            if not self._reserve(r):
                break                      # arrival order: later requests wait behind it
            pending.popleft()
            r.admitted = now
            r.stage = 0
            self.n_active += 1
            self.ex.begin(r)
            queue.append(r)

    def _limit(self, lane):
        lim = self.ex.lane_limit(lane)
        return math.inf if lim is None else lim

    def _light_limit(self):
        """The largest work estimate that a restricted lane takes (inf: none)."""
        return min(self._limit(lane) for lane in range(self.lanes))

    def _group(self, queue, limit=math.inf):
        """The waiting requests that may share a round on a lane that takes
        work estimates up to limit: the oldest eligible one and those whose
        estimate is within group_ratio of its own (every eligible one with
        group_ratio None), in arrival order, so that a small request is not
        held until a large one in its round completes."""
        elig = [r for r in queue if self.ex.cost(r.system) <= limit]
        if not elig or self.group_ratio is None:
            return elig
        c0 = self.ex.cost(elig[0].system)
        lo, hi = c0 / self.group_ratio, c0 * self.group_ratio
        return [r for r in elig if lo <= self.ex.cost(r.system) <= hi]

    # ---------------------------------------------------------- runs
    def run(self, requests):
        """Continuous batching; returns the requests with times and results."""
        pending = deque(sorted(requests, key=lambda q: (q.arrival, q.rid)))
        queue = []        # admitted, waiting for a lane
        busy = {}         # lane -> (round handle, its requests)
        t0 = self.ex.now()
        while pending or queue or busy:
            # results of completed rounds, handed back as soon as the host sees them
            for lane in sorted(busy):
                h, batch = busy[lane]
                if self.ex.done(h):
                    t = self.ex.now() - t0
                    for r in batch:
                        r.done = t
                        self.ex.end(r)
                        self._release(r)
                    del busy[lane]
            # one reading of the clock for admission and for the idle test
            # below: a request that arrives in between waits for the next trip
            now = self.ex.now() - t0
            self._admit(pending, queue, now)
            launched = False
            # the most restricted free lanes choose first
            free = sorted((lane for lane in range(self.lanes) if lane not in busy), key=self._limit)
            for lane in free:
                if not queue:
                    break
                group = self._group(queue, self._limit(lane))
                if not group:
                    continue
                # split the group between the free lanes that may take it
                c = self.ex.cost(group[0].system)
                n_free = sum(1 for x in free if x not in busy and self._limit(x) >= c)
                k = min(self.max_batch, -(-len(group) // max(1, n_free)))
                if self.heavy_alone and c > self._light_limit():
                    k = 1
                batch = group[:k]
                for r in batch:
                    queue.remove(r)
                    r.stage = 1
                busy[lane] = (self.ex.launch(batch, lane), batch)
                self.rounds.append(len(batch))
                launched = True
            if launched:
                continue
            t_next = t0 + pending[0].arrival if pending and pending[0].arrival > now else None
            if not busy and t_next is None:
                if pending and not queue:
                    raise RuntimeError("budget accounting: an idle server cannot admit a fitting request")
                continue
            self.ex.wait(t_next, [h for h, _ in busy.values()])
        return requests

    def run_sequential(self, requests):
        """One request at a time in arrival order, plain single calls."""
        t0 = self.ex.now()
        for r in sorted(requests, key=lambda q: (q.arrival, q.rid)):
            if not self._fits_ever(r):
                r.error = "request and plan exceed the HBM budget"
                continue
            if self.ex.now() - t0 < r.arrival:
                self.ex.sleep_until(t0 + r.arrival)
            if not self._reserve(r):
                raise RuntimeError("budget accounting: an idle server cannot admit a fitting request")
            r.admitted = self.ex.now() - t0
            self.n_active += 1
            self.ex.begin(r)
            self.ex.single(r)
            r.done = self.ex.now() - t0
            self.ex.end(r)
            self._release(r)
        return requests


def summarize(requests):
    """p50 / p99 latency (ms), completed requests per second, rejections."""
    done = [r for r in requests if r.error is None and not math.isnan(r.done)]
    if not done:
        return {"completed": 0, "rejected": sum(r.error is not None for r in requests)}
    lat = np.array([r.latency for r in done])
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return {"completed": len(done), "rejected": sum(r.error is not None for r in requests),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "req_per_s": len(done) / span if span > 0 else math.inf}


# ---------------------------------------------------------------- GPU side

class GPUExecutor:
    """Runs requests on one device through the C ABI.  Plans are built at
    ``register`` (their size is then known, and the FFT plans of their Poisson
    step are built and warmed up) and stay resident until the scheduler
    unloads them.  Each lane is a device stream of default priority; E_J of
    every request is copied into a pinned host slot on its lane, so that the
    host reads it without waiting for the stream."""

    N_SLOTS = 4096

    def __init__(self, device=0, precision="fp64", keep_results=False, lanes=2, light_fraction=1.0 / 3.0):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        self.device = device
        self.precision = precision
        self.keep = keep_results
        self.systems = {}
        self.plans = {}         # key -> (GPW, its Poisson step)
        self.sizes = {}         # key -> plan bytes
        self.req_sizes = {}     # key -> {kind: bytes}
        self.n_occ = {}
        self.costs = {}         # key -> work estimate
        self.n_lanes = int(lanes)
        self.light_fraction = light_fraction
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(lanes)]
        self.pinned = torch.zeros(self.N_SLOTS, dtype=torch.float64, pin_memory=True)
        self.free_slots = list(range(self.N_SLOTS - 1, -1, -1))

    def register(self, key, system, resident=True):
        from .gpw import GPW
        self.systems[key] = system
        g = GPW(system, precision=self.precision, device=self.device)
        p = g.poisson()
        # the first FFT of a mesh size builds (and compiles) its FFT plans,
        # which can take seconds: do it here, not in a request's latency
        p.solve([self.torch.zeros(tuple(m), dtype=self.torch.float64, device=self.dev) for m in g.meshes])
        info = g.info
        ngrid = sum(int(np.prod(m)) for m in info["mesh"])
        # gpw_poisson's spectra; its FFT work area is bounded by the same size
        poisson_bytes = 2 * int(info["poisson_scratch_bytes"])
        self.sizes[key] = int(info["device_bytes"])
        n2 = 8 * info["n_ao"] ** 2
        grids = 8 * ngrid
        # the library's own scratch of each operation (packed D of the collocation;
        # block-ordered potentials, with their periodic column extension, of the
        # integration and the gradient; the symmetrised D of the gradient)
        scr_rho, scr_mat, scr_grad = (int(x) for x in info["scratch_bytes"][:3])
        # D, the level densities and the potentials, the Poisson step's spectra
        # and FFT work area, the output, and the scratch of both stages (a
        # batch's collocation and second stage are enqueued back to back, so
        # their stream-ordered scratch can be live together)
        common = n2 + 2 * grids + poisson_bytes
        self.req_sizes[key] = {FOCK: common + n2 + scr_rho + scr_mat,
                               GRAD: common + 24 * info["natm"] + scr_rho + scr_grad}
        self.n_occ[key] = system.n_occ
        self.costs[key] = float(info["flops_rho_exec"] + info["flops_mat_exec"])
        if resident:
            self.plans[key] = (g, p)
        else:
            g.close()
        return self.sizes[key]

    def plan_bytes(self, key):
        return self.sizes[key]

    def request_bytes(self, key, kind):
        return self.req_sizes[key][kind]

    def cost(self, key):
        """Work estimate of a request on this system: the plan's FP64 work
        of eval_rho and eval_mat."""
        return self.costs[key]

    def lane_limit(self, lane):
        """Largest work estimate a lane takes: lane 0 any, the others the
        light requests (up to light_fraction of the largest registered
        system's), so that heavy requests run one round at a time, in arrival
        order, and light ones beside them."""
        if lane == 0 or self.light_fraction is None:
            return None
        return self.light_fraction * max(self.costs.values())

    def load(self, key):
        if key not in self.plans:
            from .gpw import GPW
            g = GPW(self.systems[key], precision=self.precision, device=self.device)
            self.plans[key] = (g, g.poisson())

    def unload(self, key):
        g, _ = self.plans.pop(key)
        self.torch.cuda.synchronize(self.dev)
        g.close()

    def density(self, key, seed):
        """D = C C^T, C an n_ao x n_occ N(0,1) matrix drawn on the device (on
        the current stream)."""
        torch = self.torch
        g, _ = self.plans[key]
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(seed)
        C = torch.randn((g.n_ao, self.n_occ[key]), dtype=torch.float64, device=self.dev, generator=gen)
        return (C @ C.T).contiguous()

    def begin(self, r):
        r.state = {"slot": self.free_slots.pop()}

    def _first_stage_inputs(self, r):
        g, _ = self.plans[r.system]
        r.state["D"] = self.density(r.system, r.seed)
        r.state["rho"] = g.new_grids()

    def _finish_poisson(self, r):
        _, p = self.plans[r.system]
        v, e = p.solve_async(r.state["rho"])
        r.state["v"] = v
        del r.state["rho"]
        # E_J to the request's pinned host slot, in stream order
        slot = r.state["slot"]
        self.pinned[slot:slot + 1].copy_(e, non_blocking=True)

    def _output(self, r):
        torch = self.torch
        g, _ = self.plans[r.system]
        shape = (g.n_ao, g.n_ao) if r.kind == FOCK else (g.natm, 3)
        r.state["out"] = torch.empty(shape, dtype=torch.float64, device=self.dev)
        return r.state["out"]

    def _second_stage(self, r):
        from . import _lib
        g, _ = self.plans[r.system]
        out = self._output(r)
        if r.kind == FOCK:
            return dict(plan=g.plan, op=_lib.GPW_OP_MAT, v=r.state["v"], out=out)
        return dict(plan=g.plan, op=_lib.GPW_OP_GRAD, D=r.state["D"], v=r.state["v"], out=out)

    def launch(self, batch, lane):
        """Enqueue the batch's round on the lane's stream: its density matrices
        and grids, one collocation batch, the Poisson steps, one integration /
        gradient batch; returns the event recorded at the round's end."""
        from . import _lib
        torch = self.torch
        st = self.streams[lane]
        with torch.cuda.stream(st):
            for r in batch:
                self._first_stage_inputs(r)
            tasks = []
            for r in batch:
                g, _ = self.plans[r.system]
                tasks.append(dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=r.state["D"], rho=r.state["rho"]))
            _lib.gpw_eval_batch(tasks)
            for r in batch:
                self._finish_poisson(r)
            _lib.gpw_eval_batch([self._second_stage(r) for r in batch])
            ev = torch.cuda.Event()
            ev.record(st)
        return ev

    def done(self, ev):
        return ev.query()

    def wait(self, t_next, events, tick=5e-5):
        """Until an event has completed or the clock reaches t_next (None: no
        arrival pending), polling every tick seconds."""
        while True:
            if any(ev.query() for ev in events):
                return
            now = time.perf_counter()
            if t_next is not None and now >= t_next:
                return
            time.sleep(tick if t_next is None else max(0.0, min(tick, t_next - now)))

    def single(self, r):
        """The plain calls of one request on the current stream, then a device
        synchronisation."""
        g, _ = self.plans[r.system]
        self._first_stage_inputs(r)
        g.rho(r.state["D"], out=r.state["rho"])
        self._finish_poisson(r)
        out = self._output(r)
        if r.kind == FOCK:
            g.mat(r.state["v"], out=out)
        else:
            g.grad(r.state["D"], r.state["v"], out=out)
        self.torch.cuda.synchronize(self.dev)

    def end(self, r):
        key = "J" if r.kind == FOCK else "grad"
        slot = r.state["slot"]
        r.result = {"E_J": float(self.pinned[slot])}
        self.free_slots.append(slot)
        if self.keep:
            r.result[key] = r.state["out"]
        r.state = {}

    def now(self):
        return time.perf_counter()

    def sleep_until(self, t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
