"""Continuous-batching request loop for FIND solves (serving).

Requests -- one mesh (Nx, Ny, stencil) with its Hamiltonian, self-energies and
a list of energies -- arrive over time.  The server keeps FIND plans (tree,
sets, gather maps and their device copies) cached per mesh shape, admits a
request as soon as a slot is free and its device footprint fits the HBM
budget beside the requests already running, and runs every admitted request
on its own HIP stream, so the work of several requests overlaps on the GPU.
A request is never split and results do not depend on what else runs: every
energy is solved by the same kernels in the same order, so a result is
bit-for-bit the one the request gets when it runs alone.

The queue is FIFO (a request that does not fit blocks the ones behind it, so
large requests are not starved).  Latency = completion - arrival; the server
reports p50/p99 latency and energy-solves/s.

The scheduling logic is independent of the GPU: `Server` drives an executor
with start(slot, req) / done(slot) / finish(slot); `GpuExecutor` runs the
HIP library, `FakeExecutor` (tests) simulates durations on a fake clock.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import find


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds from the start of the trace
    Nx: int
    Ny: int
    stencil: int
    energies: np.ndarray           # complex [nE]
    H: np.ndarray                  # [nst][Ny][Nx]
    sigma: np.ndarray              # [nE][2][Nx][Nx]
    sigma_less: np.ndarray
    want_bonds: bool = False

    @property
    def nE(self) -> int:
        return int(self.energies.size)

    @property
    def key(self):
        return (self.Nx, self.Ny, self.stencil)


@dataclasses.dataclass
class Completed:
    rid: int
    arrival: float
    admitted: float
    finished: float
    nE: int
    outputs: dict | None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class PlanCache:
    """Plans per mesh shape; a plan serves one request at a time (it owns the
    workspace of its solves).  Idle plans are kept (device state included)
    until the cached bytes would exceed the limit, then the least recently
    used are destroyed."""

    def __init__(self, precision: int, plan_budget: int, limit_bytes: int, symmetric: bool = False):
        self.precision = precision
        self.symmetric = symmetric
        self.plan_budget = plan_budget
        self.limit = limit_bytes
        self.idle = collections.OrderedDict()   # id(plan) -> (key, plan, bytes)
        self.created = 0

    def take(self, key):
        for pid, (k, plan, nbytes) in self.idle.items():
            if k == key:
                del self.idle[pid]
                return plan
        self.created += 1
        return find.Plan(*key, precision=self.precision, workspace_budget=self.plan_budget,
                         symmetric=self.symmetric)

    def give(self, key, plan, nbytes: int, inflight_bytes: int):
        self.idle[id(plan)] = (key, plan, nbytes)
        self.idle.move_to_end(id(plan))
        while self.idle and self.cached_bytes() + inflight_bytes > self.limit:
            _, (_, old, _) = self.idle.popitem(last=False)
            old.close()

    def cached_bytes(self) -> int:
        return sum(v[2] for v in self.idle.values())


class GpuExecutor:
    """Runs requests through the HIP library, one stream per slot."""

    def __init__(self, n_slots: int, precision: int = find.PREC_FP64, plan_budget: int = 16 << 30,
                 cache_limit: int = 96 << 30, device: str = "cuda", keep_outputs: bool = True,
                 symmetric: bool = False):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(n_slots)]
        self.cache = PlanCache(precision, plan_budget, cache_limit, symmetric)
        self.running = [None] * n_slots
        self.keep_outputs = keep_outputs

    def footprint(self, req: Request) -> int:
        """Device bytes of the request: its plan's footprint for nE energies,
        or what the cached plan already holds if that is more (a plan's
        buffers only grow), plus its inputs and outputs."""
        plan = self.cache.take(req.key)
        fp = max(plan.footprint(req.nE, req.want_bonds), getattr(plan, "held_bytes", 0))
        self.cache.give(req.key, plan, fp, 0)
        io = req.sigma.nbytes * 2 + req.H.nbytes + req.energies.nbytes + 2 * req.nE * req.Nx * req.Ny * 16
        if req.want_bonds:
            io += req.nE * find.n_bonds(req.Nx, req.Ny, req.stencil) * 40
        return fp + io

    def start(self, slot: int, req: Request, footprint: int) -> None:
        torch = self.torch
        plan = self.cache.take(req.key)
        plan.held_bytes = max(getattr(plan, "held_bytes", 0), plan.footprint(req.nE, req.want_bonds))
        s = self.streams[slot]
        with torch.cuda.stream(s):
            t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory().to(self.dev, non_blocking=True)
            E, H, S, SL = t(req.energies), t(req.H), t(req.sigma), t(req.sigma_less)
            nb = find.n_bonds(req.Nx, req.Ny, req.stencil)
            out = dict(diag_G=torch.empty((req.nE, req.Ny, req.Nx), dtype=torch.complex128, device=self.dev),
                       diag_Gless=torch.empty((req.nE, req.Ny, req.Nx), dtype=torch.complex128, device=self.dev))
            if req.want_bonds:
                out.update(bond_G=torch.empty((req.nE, nb), dtype=torch.complex128, device=self.dev),
                           bond_Gless=torch.empty((req.nE, nb), dtype=torch.complex128, device=self.dev),
                           bond_J=torch.empty((req.nE, nb), dtype=torch.float64, device=self.dev))
            find.solve(plan, E, H, S, SL, out["diag_G"], out["diag_Gless"], out.get("bond_G"),
                       out.get("bond_Gless"), out.get("bond_J"), stream=s)
            host = {k: torch.empty(v.shape, dtype=v.dtype, pin_memory=True) for k, v in out.items()}
            for k in out:
                host[k].copy_(out[k], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        self.running[slot] = (req, plan, footprint, ev, (E, H, S, SL, out), host)

    def done(self, slot: int) -> bool:
        return self.running[slot][3].query()

    def finish(self, slot: int, inflight_bytes: int):
        req, plan, footprint, ev, _, host = self.running[slot]
        ev.synchronize()
        find.sync_status(plan, self.streams[slot])
        self.running[slot] = None
        self.cache.give(req.key, plan, footprint, inflight_bytes)
        return {k: v.numpy() for k, v in host.items()} if self.keep_outputs else None


class Server:
    """FIFO continuous batching over `n_slots` concurrent requests with an HBM
    budget on the summed footprints of the requests in flight."""

    def __init__(self, executor, n_slots: int, hbm_budget: int, clock=time.perf_counter):
        self.ex = executor
        self.n_slots = n_slots
        self.budget = hbm_budget
        self.clock = clock
        self.queue = collections.deque()
        self.slot_req = [None] * n_slots
        self.inflight = 0
        self.max_inflight_bytes = 0
        self.max_concurrent = 0
        self.done = []
        self.t0 = None

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> None:
        fp = self.ex.footprint(req)
        if fp > self.budget:
            raise ValueError(f"request {req.rid} needs {fp} bytes, more than the HBM budget {self.budget}")
        self.queue.append((req, fp))

    def _admit(self) -> None:
        while self.queue:
            free = [i for i in range(self.n_slots) if self.slot_req[i] is None]
            if not free:
                return
            req, fp = self.queue[0]
            if self.inflight + fp > self.budget:
                return                      # FIFO: wait for memory
            self.queue.popleft()
            slot = free[0]
            self.inflight += fp
            self.max_inflight_bytes = max(self.max_inflight_bytes, self.inflight)
            self.slot_req[slot] = (req, fp, self.now())
            self.ex.start(slot, req, fp)
            self.max_concurrent = max(self.max_concurrent, sum(r is not None for r in self.slot_req))

    def _reap(self) -> int:
        n = 0
        for i in range(self.n_slots):
            if self.slot_req[i] is not None and self.ex.done(i):
                req, fp, admitted = self.slot_req[i]
                self.inflight -= fp
                outputs = self.ex.finish(i, self.inflight)
                self.slot_req[i] = None
                self.done.append(Completed(req.rid, req.arrival, admitted, self.now(), req.nE, outputs))
                n += 1
        return n

    def run(self, trace, idle_sleep: float = 2e-4) -> list:
        """Serve `trace` (requests sorted by arrival time) in real time."""
        pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
        self.t0 = self.clock()
        while pending or self.queue or any(r is not None for r in self.slot_req):
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            self._reap()
            self._admit()
            if not self._reap() and idle_sleep:
                time.sleep(idle_sleep)
        return self.done

    def stats(self) -> dict:
        lat = np.array([c.latency for c in self.done])
        span = max(c.finished for c in self.done) - min(c.arrival for c in self.done)
        return {"requests": len(self.done), "energy_solves": int(sum(c.nE for c in self.done)),
                "solves_per_s": float(sum(c.nE for c in self.done) / span),
                "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
                "makespan_s": float(span), "max_concurrent": self.max_concurrent,
                "max_inflight_bytes": int(self.max_inflight_bytes)}


def poisson_trace(n: int, rate: float, seed: int = 0, sizes=(32, 64, 128, 256), max_energies: int = 64,
                  stencils=(5, 9), want_bonds: bool = False) -> list:
    """Requests with exponential inter-arrival times (mean 1/rate); Nx uniform
    in `sizes`, Ny in {Nx, 2 Nx}, stencil uniform, 1..max_energies energies
    i.i.d. uniform in [-3.5, 3.5] + 1e-6 i (seed 1000 + request id)."""
    from . import inputs
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate)
        Nx = int(rng.choice(sizes))
        Ny = Nx * int(rng.choice([1, 2]))
        st = int(rng.choice(stencils))
        nE = int(rng.integers(1, max_energies + 1))
        p = inputs.random_problem(Nx, Ny, st, nE, seed=1000 + rid)
        out.append(Request(rid, t, Nx, Ny, st, p["energies"], p["H"], p["sigma"], p["sigma_less"], want_bonds))
    return out
