"""Serving: continuous batching of Fock-build and gradient requests.

A request names a resident system (its plan stays on the device between
requests) and carries a density matrix D.  A Fock request returns the
Coulomb matrix J = eval_mat(v_H) and E_J; a gradient request returns
dE_J/dR = eval_grad(D, v_H) and E_J, where v_H is the Hartree potential of
rho = eval_rho(D) from the multigrid Poisson step.

The scheduler runs rounds.  In every round one ``gpw_eval_batch`` call
carries the collocation task of every request admitted since the last round
and the integration (or gradient) task of every request that finished its
collocation in the previous round, so requests of different systems and
sizes share the same launches; after the batch the Poisson step of the new
requests runs.  A request therefore completes in two rounds, or in one when
no other request is waiting as the round starts (then the new requests' second
stage follows in the same round and there is nothing to batch it with anyway).
Requests that
arrive while a round is on the device are admitted at the start of the next
round, in arrival order, as long as the number of requests starting their
first stage in the round stays within ``max_active`` and their device memory
(plus that of their plan, when it is not resident) fits the HBM budget; idle plans are evicted least
recently used first to make room.  A request that can never fit is
rejected.

``run_sequential`` is the baseline: the same requests, one at a time in
arrival order, with the plain single calls.

The scheduler talks to an executor (``GPUExecutor`` here; tests use a
simulated one) through: register, plan_bytes, request_bytes, load, unload,
begin, round, single, end, now, sleep_until.
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
    def __init__(self, executor, budget_bytes, max_active=16):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.used = 0
        self.resident = OrderedDict()     # key -> plan bytes, least recently used first
        self.users = {}                   # key -> active requests on that plan
        self.rounds = []                  # per round: (n collocation tasks, n integration tasks)

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

    def _admit(self, pending, active, now):
        # at the start of a round every active request is in its second stage
        # and leaves with this round: the slots limit the new (first-stage) ones
        new = sum(1 for r in active if r.stage == 0)
        while pending and pending[0].arrival <= now and new < self.max_active:
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
            self.ex.begin(r)
            active.append(r)
            new += 1

    # ---------------------------------------------------------- runs
    def run(self, requests):
        """Continuous batching; returns the requests with times and results."""
        pending = deque(sorted(requests, key=lambda q: (q.arrival, q.rid)))
        active = []
        t0 = self.ex.now()
        while pending or active:
            self._admit(pending, active, self.ex.now() - t0)
            if not active:
                if pending:
                    self.ex.sleep_until(t0 + pending[0].arrival)
                continue
            s0 = [r for r in active if r.stage == 0]
            s1 = [r for r in active if r.stage == 1]
            # nobody waiting: the new requests finish in this round too
            fuse = not (pending and pending[0].arrival <= self.ex.now() - t0)
            t_s1 = self.ex.round(s0, s1, fuse)
            now = self.ex.now() - t0
            self.rounds.append((len(s0), len(s1)))
            for r in s1 + (s0 if fuse else []):
                # second-stage results are complete when the round's batch is,
                # before the new requests' Poisson steps
                r.done = t_s1 - t0 if (t_s1 is not None and r.stage == 1) else now
                self.ex.end(r)
                self._release(r)
                active.remove(r)
            if not fuse:
                for r in s0:
                    r.stage = 1
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
    unloads them."""

    def __init__(self, device=0, precision="fp64", keep_results=False):
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
        # D, the level densities and then potentials, the Poisson step's
        # spectra and FFT work area; the collocation's and the second stage's
        # scratch never coexist within one request
        common = n2 + 2 * grids + poisson_bytes
        self.req_sizes[key] = {FOCK: common + n2 + max(scr_rho, scr_mat),
                               GRAD: common + 24 * info["natm"] + max(scr_rho, scr_grad)}
        self.n_occ[key] = system.n_occ
        if resident:
            self.plans[key] = (g, p)
        else:
            g.close()
        return self.sizes[key]

    def plan_bytes(self, key):
        return self.sizes[key]

    def request_bytes(self, key, kind):
        return self.req_sizes[key][kind]

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
        """D = C C^T, C an n_ao x n_occ N(0,1) matrix drawn on the device."""
        torch = self.torch
        g, _ = self.plans[key]
        gen = torch.Generator(device=self.dev)
        gen.manual_seed(seed)
        C = torch.randn((g.n_ao, self.n_occ[key]), dtype=torch.float64, device=self.dev, generator=gen)
        return (C @ C.T).contiguous()

    def begin(self, r):
        g, _ = self.plans[r.system]
        r.state = {"D": self.density(r.system, r.seed), "rho": g.new_grids()}

    def _finish_poisson(self, r):
        _, p = self.plans[r.system]
        v, e = p.solve_async(r.state["rho"])
        r.state["v"] = v
        r.state["E_J"] = e          # device scalar, read when the request ends
        del r.state["rho"]

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

    def round(self, s0, s1, finish_new=False):
        """The second stage of s1 as one batch, then the collocation of s0 as
        another, queued back to back, then the Poisson steps of s0 (and, with
        finish_new, their second stage).  Returns the time at which the s1
        results were complete (None without s1), read from a stream event so
        that the s0 work is not held back by a synchronisation."""
        from . import _lib
        torch = self.torch
        if finish_new and len(s0) == 1 and not s1:
            # a lone request: the plain calls, as the one-at-a-time server makes them
            self.single(s0[0])
            return None
        t_h0 = self.now()
        ev0 = ev1 = None
        if s1:
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            _lib.gpw_eval_batch([self._second_stage(r) for r in s1])
            ev1.record()
        if s0:
            tasks = []
            for r in s0:
                g, _ = self.plans[r.system]
                tasks.append(dict(plan=g.plan, op=_lib.GPW_OP_RHO, D=r.state["D"], rho=r.state["rho"]))
            _lib.gpw_eval_batch(tasks)
        for r in s0:
            self._finish_poisson(r)
        if finish_new and s0:
            _lib.gpw_eval_batch([self._second_stage(r) for r in s0])
        torch.cuda.synchronize(self.dev)
        return t_h0 + ev0.elapsed_time(ev1) * 1e-3 if s1 else None

    def single(self, r):
        g, _ = self.plans[r.system]
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
        r.result = {"E_J": float(r.state["E_J"].item())}
        if self.keep:
            r.result[key] = r.state["out"]
        r.state = {}

    def now(self):
        return time.perf_counter()

    def sleep_until(self, t):
        dt = t - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
