"""Continuous-batching request server for ISDC time integration.

Requests (an initial state, a problem, step size, number of steps and a
tolerance) arrive over time.  The server keeps one batch per spatial
dimension, each advanced on a stream of its own; a request is admitted into a
free slot as soon as its device memory (plan workspace + state) fits under the
HBM budget (``choose_admissions``: first come first served, and the oldest
request that does not fit reserves its memory, so later and smaller requests
can only fill what is left beside it), its state then stays resident on the
device between sweeps, every ``advance`` moves all admitted requests of a
batch by one sweep in shared kernel launches -- the batches of the two
dimensions at the same time, from two host threads on two streams -- and a
request leaves (freeing its slot and memory) when its last step has converged
or it has failed.  Requests therefore join and leave at sweep boundaries
while others are on the GPU.

All computation is in the HIP library; this module is scheduling and
bookkeeping only.
"""
from __future__ import annotations

import math
import sys
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as A
from .isdc import Batch, Plan, make_params, make_problem, workspace_bytes  # noqa: F401


# device copies of request initial states, shared by the runs of one process
_U0_DEVICE: dict = {}


@dataclass
class Request:
    rid: int
    dim: int
    n: int
    nu: float
    fe_kind: int
    modes: list                 # u_0 = scale * sum of these sine modes
    dt: float
    nsteps: int
    sdc_tol: float
    M: int = 3
    node_kind: int = A.NODES_LOBATTO
    arrival: float = 0.0        # seconds after the start of the run
    scale: float = 1.0
    # filled by the server
    admitted: float = math.nan
    finished: float = math.nan
    status: str = ""
    result: torch.Tensor | None = None
    sweeps_last_step: int = 0
    solo: bool = True           # ran on a plan of its own (False: in a batch slot)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival

    @property
    def u0(self) -> np.ndarray:
        """Initial state on the host (float64, shape (n,)*dim)."""
        from . import workloads as W
        return W.sine_field(self.n, self.dim, self.modes) * self.scale

    def u0_device(self) -> torch.Tensor:
        """A fresh device copy of the initial state (equal to u0 bit for bit;
        built on the device once per process and cached)."""
        from . import workloads as W
        key = (self.dim, self.n, self.scale, tuple((float(a), tuple(w)) for a, w in self.modes))
        t = _U0_DEVICE.get(key)
        if t is None:
            t = W.sine_field_device(self.n, self.dim, self.modes) * self.scale
            torch.cuda.current_stream().synchronize()  # other threads' streams read it later
            _U0_DEVICE[key] = t
        return t.clone()

    def params(self, precision: int, vcycles: int) -> dict:
        """Plan parameters, the same on a solo lane and in a batch slot: 2D
        requests take weighted-Jacobi V(3,3) cycles on the fused row kernels
        (fewer sweeps than red-black V(1,1), most of all for the reaction-
        diffusion requests), 3D requests red-black V(1,1)."""
        p = dict(node_kind=self.node_kind, M=self.M, sdc_tol=self.sdc_tol, precision=precision,
                 vcycles=vcycles, max_sweeps=200)
        if self.dim == 2:
            p.update(smoother=A.SMOOTH_JACOBI, nu_pre=3, nu_post=3)
        return p

    def device_bytes(self, precision: int, vcycles: int) -> int:
        key = (precision, vcycles)
        if getattr(self, "_bytes_key", None) != key:
            prob = make_problem(self.dim, self.n, self.nu, self.fe_kind)
            par = make_params(**self.params(precision, vcycles))
            self._bytes = workspace_bytes(prob, par) + self.n ** self.dim * 8
            self._bytes_key = key
        return self._bytes


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


def choose_admissions(waiting, need, used: int, budget: int, free_slots: dict) -> list:
    """Requests of `waiting` (in arrival order) to admit now: each in turn if a
    slot of its dimension is free and its memory fits in the budget.  The
    first request that cannot be admitted reserves its memory: every later one
    must then fit beside that reservation, so the oldest waiting request gets
    the memory that frees up and cannot be passed over indefinitely by smaller
    ones.  `need(r)` gives a request's bytes; `free_slots` maps a dimension to
    its number of free slots."""
    slots = dict(free_slots)
    mem = used
    reserve = 0
    blocked = False
    out = []
    for r in waiting:
        b = need(r)
        if slots.get(r.dim, 0) > 0 and mem + b + reserve <= budget:
            out.append(r)
            mem += b
            slots[r.dim] -= 1
        elif not blocked:
            blocked = True
            reserve = b
    return out


# A request runs on a plan of its own ("solo": isdc_step on its own stream,
# from a worker thread) when it is large -- 2D grids of 511^2 and up, 3D of
# 127^3 and up, where the single-instance kernels (row tiles, z-marched
# planes) beat the batch's generic ones and one instance fills much of the
# chip -- or when no batch slot of its dimension is running, so that a
# request arriving at an idle server is not slowed by the batch machinery.
def runs_solo(req, batch_running: int) -> bool:
    big = (req.dim == 2 and req.n >= 511) or (req.dim == 3 and req.n >= 127)
    return big or batch_running == 0


class Server:
    """One batch per dimension plus `solo_workers` solo lanes; admission by
    slots and HBM budget (bytes)."""

    def __init__(self, hbm_budget: int, slots_per_batch: int = 64, precision: int = A.PREC_MIXED,
                 vcycles: int = 2, dims=(2, 3), solo_workers: int = 2):
        self.budget = int(hbm_budget)
        self.precision = precision
        self.vcycles = vcycles
        self.batches = {d: Batch(slots_per_batch, d, precision=precision, vcycles=vcycles) for d in dims}
        # one stream per batch and per solo lane (default priority), each driven from a thread of its own
        self.streams = {d: torch.cuda.Stream() for d in dims}
        self.pool = ThreadPoolExecutor(max_workers=len(dims))
        self.solo_pool = ThreadPoolExecutor(max_workers=max(1, solo_workers)) if solo_workers > 0 else None
        self.solo_streams = [torch.cuda.Stream() for _ in range(solo_workers)]
        self.solo_free = list(range(solo_workers))
        self.solo_running = {}  # future -> (request, bytes, lane)
        self.free = {d: list(range(slots_per_batch)) for d in dims}
        self.running = {d: {} for d in dims}   # slot -> (request, bytes)
        self.used = 0

    def __del__(self):
        try:
            self.pool.shutdown(wait=False)
            if self.solo_pool is not None:
                self.solo_pool.shutdown(wait=False)
        except Exception:
            pass

    def _solo_job(self, req: Request, stream, t0: float, clock):
        """All steps of one request on its own plan and stream (a worker thread)."""
        with torch.cuda.stream(stream):
            p = Plan(req.dim, req.n, req.nu, req.fe_kind, **req.params(self.precision, self.vcycles))
            u = req.u0_device()
            status, sweeps = "ok", 0
            for _ in range(req.nsteps):
                st = p.step(u, req.dt, stream=stream)
                sweeps = st.sweeps
                if st.status != "ok":
                    status = st.status
                    break
            stream.synchronize()
        return status, u, sweeps, clock() - t0

    def _admit_solo(self, req: Request, now: float, t0: float, clock) -> None:
        need = self._need(req)
        lane = self.solo_free.pop(0)
        req.admitted = now
        req.solo = True
        f = self.solo_pool.submit(self._solo_job, req, self.solo_streams[lane], t0, clock)
        self.solo_running[f] = (req, need, lane)
        self.used += need

    def _reap_solo(self, stats: ServeStats) -> bool:
        done = [f for f in self.solo_running if f.done()]
        for f in done:
            req, need, lane = self.solo_running.pop(f)
            status, u, sweeps, finished = f.result()
            req.finished = finished
            req.status = status
            req.result = u
            req.sweeps_last_step = sweeps
            if status == "ok":
                stats.completed += 1
                stats.latencies.append(req.latency)
            else:
                stats.failed += 1
            self.solo_free.append(lane)
            self.used -= need
        return bool(done)

    def _need(self, req: Request) -> int:
        need = req.device_bytes(self.precision, self.vcycles)
        if need > self.budget:
            raise ValueError(f"request {req.rid} needs {need} bytes, more than the whole budget")
        return need

    def _admit(self, req: Request, now: float) -> bool:
        need = self._need(req)
        d = req.dim
        if not self.free[d] or self.used + need > self.budget:
            return False
        slot = self.free[d].pop(0)
        par = req.params(self.precision, self.vcycles)
        ws = torch.empty(need - req.n ** req.dim * 8, dtype=torch.uint8, device="cuda")
        u = req.u0_device()
        self.batches[d].set(slot, u, req.dt, req.nsteps, req.nu, req.fe_kind, workspace=ws, **par)
        req.admitted = now
        req.solo = False
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

    def serve(self, requests: list[Request], clock=time.perf_counter, log_every: int = 0) -> ServeStats:
        """Run until every request has finished.  Arrival times are honoured in
        wall-clock time: a request is admissible once its arrival has passed.
        log_every > 0 prints a progress line to stderr every that many finished requests."""
        queue = sorted(requests, key=lambda r: r.arrival)
        stats = ServeStats()
        t0 = clock()
        i = 0
        waiting: list[Request] = []
        while i < len(queue) or waiting or any(self.running[d] for d in self.running) or self.solo_running:
            now = clock() - t0
            while i < len(queue) and queue[i].arrival <= now:
                waiting.append(queue[i])
                i += 1
            before = stats.completed + stats.failed
            self._reap_solo(stats)
            admit = choose_admissions(waiting, self._need, self.used, self.budget,
                                      {d: len(f) for d, f in self.free.items()})
            for r in admit:
                if self.solo_free and runs_solo(r, len(self.running[r.dim])):
                    self._admit_solo(r, now, t0, clock)
                else:
                    ok = self._admit(r, now)
                    assert ok
            if admit:
                chosen = set(id(r) for r in admit)
                waiting = [r for r in waiting if id(r) not in chosen]
                # the states were uploaded on the current stream; the batch streams start after them
                torch.cuda.current_stream().synchronize()
            stats.peak_bytes = max(stats.peak_bytes, self.used)
            stats.peak_concurrency = max(stats.peak_concurrency,
                                         sum(len(v) for v in self.running.values()) + len(self.solo_running))
            # one sweep of every batch with running slots, the batches side by side
            live = [d for d in self.batches if self.running[d]]
            futures = [self.pool.submit(self.batches[d].advance, self.streams[d]) for d in live]
            for f in futures:
                f.result()
            stats.advances += len(live)
            busy = bool(live)
            for d in live:
                self._reap(d, clock() - t0, stats)
            done = stats.completed + stats.failed
            if log_every and done // log_every > before // log_every:
                print(f"[serve] {done}/{len(queue)} requests finished at {clock() - t0:.1f} s",
                      file=sys.stderr, flush=True)
            if not busy:
                # idle until the next arrival or the next solo request's end
                delay = 0.05
                if i < len(queue):
                    delay = min(delay, queue[i].arrival - (clock() - t0))
                if self.solo_running:
                    delay = min(delay, 0.0005)
                if delay > 0:
                    time.sleep(delay)
        stats.makespan = clock() - t0
        return stats


def serve_sequential(requests: list[Request], precision: int = A.PREC_MIXED, vcycles: int = 2,
                     clock=time.perf_counter, log_every: int = 0) -> ServeStats:
    """Baseline: requests served one after another (FIFO) with isdc_step."""
    queue = sorted(requests, key=lambda r: r.arrival)
    stats = ServeStats()
    t0 = clock()
    for k, req in enumerate(queue):
        if log_every and k and k % log_every == 0:
            print(f"[serve-seq] {k}/{len(queue)} requests finished at {clock() - t0:.1f} s", file=sys.stderr,
                  flush=True)
        now = clock() - t0
        if req.arrival > now:
            time.sleep(req.arrival - now)
        req.admitted = clock() - t0
        p = Plan(req.dim, req.n, req.nu, req.fe_kind, **req.params(precision, vcycles))
        u = req.u0_device()
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
        out.append(Request(rid=rid, dim=dim, n=n, nu=1.0 if heat else 0.1, fe_kind=0 if heat else 1, modes=modes,
                           dt=1e-3, nsteps=steps, sdc_tol=tol, M=M, arrival=t, scale=1.0 if heat else 3.0))
    return out
