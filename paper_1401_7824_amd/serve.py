"""Continuous-batching request server for ISDC time integration.

Requests (an initial state, a problem, step size, number of steps and a
tolerance) arrive over time.  The server keeps one batch per spatial
dimension; a request is admitted into a free slot as soon as its device memory
(plan workspace + state) fits under the HBM budget, its state then stays
resident on the device between sweeps, every ``advance`` moves all admitted
requests of a batch by one sweep in shared kernel launches, and a request
leaves (freeing its slot and memory) when its last step has converged or it
has failed.  Requests therefore join and leave at sweep boundaries while
others are on the GPU.

All computation is in the HIP library; this module is scheduling and
bookkeeping only.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as A
from .isdc import Batch, Plan, make_params, make_problem, workspace_bytes


@dataclass
class Request:
    rid: int
    dim: int
    n: int
    nu: float
    fe_kind: int
    u0: np.ndarray
    dt: float
    nsteps: int
    sdc_tol: float
    M: int = 3
    node_kind: int = A.NODES_LOBATTO
    arrival: float = 0.0        # seconds after the start of the run
    # filled by the server
    admitted: float = math.nan
    finished: float = math.nan
    status: str = ""
    result: torch.Tensor | None = None
    sweeps_last_step: int = 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    def params(self, precision: int, vcycles: int) -> dict:
        return dict(node_kind=self.node_kind, M=self.M, sdc_tol=self.sdc_tol, precision=precision,
                    vcycles=vcycles, max_sweeps=200)

    def device_bytes(self, precision: int, vcycles: int) -> int:
        prob = make_problem(self.dim, self.n, self.nu, self.fe_kind)
        return workspace_bytes(prob, make_params(**self.params(precision, vcycles))) + self.n ** self.dim * 8


@dataclass
class ServeStats:
    completed: int = 0
    failed: int = 0
    makespan: float = 0.0
    latencies: list = field(default_factory=list)
    peak_bytes: int = 0
    peak_concurrency: int = 0
    advances: int = 0

    def summary(self) -> dict:
        lat = np.array(self.latencies) if self.latencies else np.array([math.nan])
        return dict(completed=self.completed, failed=self.failed, makespan_s=round(self.makespan, 4),
                    throughput_req_s=round(self.completed / self.makespan, 3) if self.makespan > 0 else None,
                    p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 3),
                    p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 3),
                    mean_ms=round(float(lat.mean()) * 1e3, 3), peak_bytes=self.peak_bytes,
                    peak_concurrency=self.peak_concurrency, batch_sweeps=self.advances)


class Server:
    """One batch per dimension, admission by slots and HBM budget (bytes)."""

    def __init__(self, hbm_budget: int, slots_per_batch: int = 64, precision: int = A.PREC_MIXED,
                 vcycles: int = 2, dims=(2, 3)):
        self.budget = int(hbm_budget)
        self.precision = precision
        self.vcycles = vcycles
        self.batches = {d: Batch(slots_per_batch, d, precision=precision, vcycles=vcycles) for d in dims}
        self.free = {d: list(range(slots_per_batch)) for d in dims}
        self.running = {d: {} for d in dims}   # slot -> (request, bytes)
        self.used = 0

    def _admit(self, req: Request, now: float) -> bool:
        need = req.device_bytes(self.precision, self.vcycles)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} bytes, more than the whole budget")
        d = req.dim
        if not self.free[d] or self.used + need > self.budget:
            return False
        slot = self.free[d].pop(0)
        par = req.params(self.precision, self.vcycles)
        ws = torch.empty(need - req.n ** req.dim * 8, dtype=torch.uint8, device="cuda")
        u = torch.from_numpy(np.ascontiguousarray(req.u0)).to("cuda")
        self.batches[d].set(slot, u, req.dt, req.nsteps, req.nu, req.fe_kind, workspace=ws, **par)
        req.admitted = now
        req.result = u
        self.running[d][slot] = (req, need, ws)
        self.used += need
        return True

    def _reap(self, d: int, now: float, stats: ServeStats):
        b = self.batches[d]
        for slot, (req, need, ws) in list(self.running[d].items()):
            state, status, steps, last = b.info(slot)
            if state == A.SLOT_FINISHED:
                req.finished = now
                req.status = status
                req.sweeps_last_step = last.sweeps
                if status == "ok":
                    stats.completed += 1
                    stats.latencies.append(req.latency)
                else:
                    stats.failed += 1
                b.release(slot)
                del self.running[d][slot]
                self.free[d].append(slot)
                self.used -= need

    def serve(self, requests: list[Request], clock=time.perf_counter) -> ServeStats:
        """Run until every request has finished.  Arrival times are honoured in
        wall-clock time: a request is admissible once its arrival has passed."""
        queue = sorted(requests, key=lambda r: r.arrival)
        stats = ServeStats()
        t0 = clock()
        i = 0
        waiting: list[Request] = []
        while i < len(queue) or waiting or any(self.running[d] for d in self.running):
            now = clock() - t0
            while i < len(queue) and queue[i].arrival <= now:
                waiting.append(queue[i])
                i += 1
            # FIFO admission while memory and slots allow (a request that does not
            # fit blocks the ones behind it of the same dimension)
            blocked = set()
            rest = []
            for r in waiting:
                if r.dim in blocked or not self._admit(r, now):
                    blocked.add(r.dim)
                    rest.append(r)
            waiting = rest
            stats.peak_bytes = max(stats.peak_bytes, self.used)
            stats.peak_concurrency = max(stats.peak_concurrency, sum(len(v) for v in self.running.values()))
            busy = False
            for d, b in self.batches.items():
                if self.running[d]:
                    b.advance()
                    stats.advances += 1
                    busy = True
                    self._reap(d, clock() - t0, stats)
            if not busy:
                # idle until the next arrival
                if i < len(queue):
                    delay = queue[i].arrival - (clock() - t0)
                    if delay > 0:
                        time.sleep(min(delay, 0.05))
        stats.makespan = clock() - t0
        return stats


def serve_sequential(requests: list[Request], precision: int = A.PREC_MIXED, vcycles: int = 2,
                     clock=time.perf_counter) -> ServeStats:
    """Baseline: requests served one after another (FIFO) with isdc_step."""
    queue = sorted(requests, key=lambda r: r.arrival)
    stats = ServeStats()
    t0 = clock()
    for req in queue:
        now = clock() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        req.admitted = clock() - t0
        p = Plan(req.dim, req.n, req.nu, req.fe_kind, **req.params(precision, vcycles))
        u = torch.from_numpy(np.ascontiguousarray(req.u0)).to("cuda")
        status = "ok"
        for _ in range(req.nsteps):
            st = p.step(u, req.dt)
            if st.status != "ok":
                status = st.status
                break
        torch.cuda.synchronize()
        req.finished = clock() - t0
        req.status = status
        req.result = u
        if status == "ok":
            stats.completed += 1
            stats.latencies.append(req.latency)
        else:
            stats.failed += 1
    stats.makespan = clock() - t0
    return stats


def make_requests(count: int, rate: float, seed: int = 5, big: bool = True) -> list[Request]:
    """Synthetic request mix: half 2D (side 127..1023), half 3D (31..255);
    half heat (nu = 1, f^E = 0), half reaction-diffusion (nu = 0.1, u - u^3);
    dt = 1e-3; Gauss-Lobatto M in {3, 5}; tolerance 1e-5 or 1e-8; 1..20
    steps; Poisson arrivals at `rate` per second.  big=False caps the sizes at
    255^2 / 63^3 and the steps at 5 (quick runs)."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        dim = 2 if rng.random() < 0.5 else 3
        k = int(rng.integers(7, 11)) if dim == 2 else int(rng.integers(5, 9))
        if not big:
            k = min(k, 8 if dim == 2 else 6)
        n = 2 ** k - 1
        heat = rng.random() < 0.5
        M = int(rng.choice([3, 5]))
        tol = float(rng.choice([1e-5, 1e-8]))
        steps = int(rng.integers(1, 21)) if big else int(rng.integers(1, 6))
        modes = W.draw_modes(dim, 8, seed=10_000 + rid, max_wave=4)
        u0 = W.sine_field(n, dim, modes) * (1.0 if heat else 3.0)
        out.append(Request(rid=rid, dim=dim, n=n, nu=1.0 if heat else 0.1, fe_kind=0 if heat else 1, u0=u0,
                           dt=1e-3, nsteps=steps, sdc_tol=tol, M=M, arrival=t))
    return out
