"""Python binding of libisdc: plans over torch-allocated device memory.

PyTorch provides device memory (the workspace and the grid arrays) and the
stream; every computation is a kernel of the HIP library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import torch

from . import _capi as A


@dataclass
class StepStats:
    status: str
    sweeps: int
    vcycles: int
    residual: float
    residual_hist: list = field(default_factory=list)
    coarse_vcycles: int = 0

    @classmethod
    def from_c(cls, st: A.Stats, rc: int) -> "StepStats":
        return cls(status=A.STATUS_NAMES.get(rc, str(rc)), sweeps=st.sweeps, vcycles=st.vcycles,
                   residual=st.residual, residual_hist=[st.residual_hist[i] for i in range(st.hist_len)],
                   coarse_vcycles=st.coarse_vcycles)


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype=None, numel=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"tensor must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def make_problem(dim, n, nu, fe_kind=A.FE_ZERO, stencil=A.STENCIL_2ND, bc=A.BC_DIRICHLET) -> A.Problem:
    return A.problem(dim, n, nu, fe_kind, stencil, bc)


def make_params(**kw) -> A.Params:
    lib = A.load()
    p = A.Params()
    A.check(lib.isdc_default_params(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, int(v) if isinstance(v, bool) else v)
    return p


def tables(node_kind: int, M: int):
    """(tau, Q, S) from the library's host-side table generator, as lists."""
    lib = A.load()
    tau = (C.c_double * M)()
    Q = (C.c_double * (M * M))()
    S = (C.c_double * (M * M))()
    A.check(lib.isdc_tables(node_kind, M, tau, Q, S))
    return list(tau), [list(Q[i * M:(i + 1) * M]) for i in range(M)], [list(S[i * M:(i + 1) * M]) for i in range(M)]


def end_weights(node_kind: int, M: int):
    """Whole-step weights b_j (integral of l_j over [0, 1]) from the library, as a list."""
    lib = A.load()
    b = (C.c_double * M)()
    A.check(lib.isdc_end_weights(node_kind, M, b))
    return list(b)


def workspace_bytes(problem: A.Problem, params: A.Params) -> int:
    lib = A.load()
    out = C.c_size_t()
    A.check(lib.isdc_workspace_bytes(C.byref(problem), C.byref(params), C.byref(out)))
    return out.value


def step_noalloc(u: torch.Tensor, dt: float, nu: float, fe_kind: int = A.FE_ZERO, stencil: int = A.STENCIL_2ND,
                 bc: int = A.BC_DIRICHLET, stream=None, **params) -> StepStats:
    """One ISDC step in place on u (float64, shape (n,)*d) through
    isdc_step_noalloc: the library's static device scratch instead of a
    workspace, so nothing is allocated on the device."""
    lib = A.load()
    dim, n = u.dim(), u.shape[0]
    prob = make_problem(dim, n, nu, fe_kind, stencil, bc)
    par = make_params(**params)
    st = A.Stats()
    rc = lib.isdc_step_noalloc(C.byref(prob), C.byref(par), _dev_ptr(u, torch.float64, n ** dim), dt,
                               _stream_handle(stream), C.byref(st))
    A.check(rc, allow=(A.E_NOT_CONVERGED, A.E_DIVERGED))
    return StepStats.from_c(st, rc)


class Plan:
    """One ISDC problem instance: the C plan plus its torch-owned workspace."""

    def __init__(self, dim: int, n: int, nu: float, fe_kind: int = A.FE_ZERO, device=None,
                 stencil: int = A.STENCIL_2ND, bc: int = A.BC_DIRICHLET, **params):
        self.lib = A.load()
        self.problem = make_problem(dim, n, nu, fe_kind, stencil, bc)
        self.params = make_params(**params)
        self.dim, self.n = dim, n
        self.periodic = bc == A.BC_PERIODIC
        self.stencil = stencil
        self.N = n ** dim
        self.shape = (n,) * dim
        nbytes = workspace_bytes(self.problem, self.params)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        A.check(self.lib.isdc_create(C.byref(self.problem), C.byref(self.params),
                                     C.c_void_p(self.workspace.data_ptr()), nbytes, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.isdc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- the time step ----
    def step(self, u: torch.Tensor, dt: float, stream=None) -> StepStats:
        """One ISDC step in place on u (float64, shape (n,)*d)."""
        st = A.Stats()
        rc = self.lib.isdc_step(self._h, _dev_ptr(u, torch.float64, self.N), dt, _stream_handle(stream),
                                C.byref(st))
        A.check(rc, allow=(A.E_NOT_CONVERGED, A.E_DIVERGED))
        return StepStats.from_c(st, rc)

    def begin(self, u0: torch.Tensor, dt: float, stream=None):
        self._u0 = u0  # must stay alive and unchanged until end()
        A.check(self.lib.isdc_begin(self._h, _dev_ptr(u0, torch.float64, self.N), dt, _stream_handle(stream)))

    def sweep(self, stream=None) -> float:
        r = C.c_double()
        A.check(self.lib.isdc_sweep(self._h, _stream_handle(stream), C.byref(r)))
        return r.value

    def end(self, out: torch.Tensor, stream=None):
        A.check(self.lib.isdc_end(self._h, _dev_ptr(out, torch.float64, self.N), _stream_handle(stream)))
        self._u0 = None

    def node_values(self, j: int, stream=None) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        A.check(self.lib.isdc_node_values(self._h, j, _dev_ptr(out), _stream_handle(stream)))
        return out

    def stats(self) -> StepStats:
        st = A.Stats()
        A.check(self.lib.isdc_get_stats(self._h, C.byref(st)))
        return StepStats.from_c(st, A.OK)

    # ---- multigrid ----
    def vcycle(self, c: float, rhs: torch.Tensor, u: torch.Tensor, ncycles: int = 1, want_residual=False,
               stream=None):
        prec = A.PREC_FP64 if u.dtype == torch.float64 else A.PREC_MIXED
        dt = torch.float64 if prec == A.PREC_FP64 else torch.float32
        res = C.c_double()
        A.check(self.lib.isdc_vcycle(self._h, c, prec, _dev_ptr(rhs, dt, self.N), _dev_ptr(u, dt, self.N),
                                     ncycles, _stream_handle(stream), C.byref(res) if want_residual else None))
        return res.value if want_residual else None

    def level_n(self, level: int) -> int:
        """Points per axis of multigrid level `level` (periodic n / 2^l, else (n+1) / 2^l - 1)."""
        return self.n >> level if self.periodic else ((self.n + 1) >> level) - 1

    def mg_op(self, op: int, level: int, c: float, a=None, b=None, out=None, stream=None):
        t = next(x for x in (a, b, out) if x is not None)
        prec = A.PREC_FP64 if t.dtype == torch.float64 else A.PREC_MIXED
        dt = torch.float64 if prec == A.PREC_FP64 or op == A.OP_EXPLICIT else torch.float32
        fine = self.level_n(level) ** self.dim
        coarse = self.level_n(level + 1) ** self.dim if self.level_n(level) > 1 else 0
        sizes = {A.OP_SMOOTH: (fine, fine, fine), A.OP_RESTRICT: (fine, fine, coarse),
                 A.OP_PROLONG: (coarse, None, fine), A.OP_COARSE: (fine, None, fine),
                 A.OP_RESIDUAL_NORM: (fine, fine, None), A.OP_EXPLICIT: (fine, None, fine)}.get(op, (None,) * 3)
        ptrs = [_dev_ptr(x, dt, sz) for x, sz in zip((a, b, out), sizes)]
        res = C.c_double()
        A.check(self.lib.isdc_mg_op(self._h, op, level, c, prec, *ptrs, _stream_handle(stream), C.byref(res)))
        return res.value

    @property
    def tile_shapes(self) -> list:
        """Tile shape of the multigrid kernels per level above the coarse tail."""
        buf = (C.c_int32 * 32)()
        nl = C.c_int32()
        A.check(self.lib.isdc_get_tile_shapes(self._h, buf, 32, C.byref(nl)))
        return list(buf[:nl.value])

    @tile_shapes.setter
    def tile_shapes(self, shapes):
        arr = (C.c_int32 * max(1, len(shapes)))(*shapes)
        A.check(self.lib.isdc_set_tile_shapes(self._h, arr, len(shapes)))

    def autotune(self, reps: int = 50, cache: bool = True, stream=None) -> list:
        """Pick the tile shape of every level by timing (isdc_autotune), or
        take the choice stored for this device and plan shape in the tuning
        cache (tuning.py); returns the shapes."""
        from . import tuning
        key = tuning.key(self) if cache else None
        if key is not None:
            saved = tuning.lookup(key)
            if saved is not None and len(saved) == len(self.tile_shapes):
                self.tile_shapes = saved
                return saved
        buf = (C.c_int32 * 32)()
        nl = C.c_int32()
        A.check(self.lib.isdc_autotune(self._h, reps, _stream_handle(stream), buf, 32, C.byref(nl)))
        shapes = list(buf[:nl.value])
        if key is not None:
            tuning.store(key, shapes)
        return shapes

    def probe_arm(self, kernel: int, level: int = 0, every: int = 1, max_samples: int = 100000):
        """Follow `kernel` on `level` inside the next steps (isdc_probe_arm)."""
        A.check(self.lib.isdc_probe_arm(self._h, kernel, level, every, max_samples))

    def probe_read(self):
        """(samples, average microseconds per launch, average algorithmic bytes per launch)
        of the launches followed since probe_arm (isdc_probe_read)."""
        n, us, b = C.c_int64(), C.c_double(), C.c_double()
        A.check(self.lib.isdc_probe_read(self._h, C.byref(n), C.byref(us), C.byref(b)))
        return n.value, us.value, b.value

    def time_kernel(self, kernel: int, level: int, c: float, precision: int, reps: int = 100, stream=None):
        """(average microseconds per launch, algorithmic bytes per launch) of one library kernel."""
        us, b = C.c_double(), C.c_double()
        A.check(self.lib.isdc_time_kernel(self._h, kernel, level, c, precision, reps, _stream_handle(stream),
                                          C.byref(us), C.byref(b)))
        return us.value, b.value


class Batch:
    """Many independent ISDC instances advanced together (one launch per sweep
    phase for all running slots).  Device memory for the batch tables and for
    every slot's plan comes from torch; the state tensors stay owned by the
    caller and are kept alive here until their slot is released."""

    def __init__(self, capacity: int, dim: int, precision: int = A.PREC_FP64, vcycles: int = 2, device=None):
        self.lib = A.load()
        self.capacity, self.dim, self.precision, self.vcycles = capacity, dim, precision, vcycles
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        nbytes = C.c_size_t()
        A.check(self.lib.isdc_batch_workspace_bytes(capacity, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        A.check(self.lib.isdc_batch_open(capacity, dim, precision, vcycles, C.c_void_p(self.workspace.data_ptr()),
                                         nbytes.value, C.byref(h)))
        self._h = h
        self._keep = [None] * capacity

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.isdc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def workspace_bytes_for(n: int, dim: int, nu: float, fe_kind: int = A.FE_ZERO, **params) -> int:
        return workspace_bytes(make_problem(dim, n, nu, fe_kind), make_params(**params))

    def set(self, slot: int, u: torch.Tensor, dt: float, nsteps: int, nu: float, fe_kind: int = A.FE_ZERO,
            workspace: torch.Tensor = None, stencil: int = A.STENCIL_2ND, bc: int = A.BC_DIRICHLET, **params):
        """Start instance (u, nu, f^E, params) in `slot` for nsteps steps of size dt.
        u (float64, shape (n,)*dim) is advanced in place."""
        n = u.shape[0]
        params.setdefault("vcycles", self.vcycles)
        params.setdefault("precision", self.precision)
        prob = make_problem(self.dim, n, nu, fe_kind, stencil, bc)
        par = make_params(**params)
        need = workspace_bytes(prob, par)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        A.check(self.lib.isdc_batch_set(self._h, slot, C.byref(prob), C.byref(par),
                                        C.c_void_p(workspace.data_ptr()), workspace.numel(),
                                        _dev_ptr(u, torch.float64, n ** self.dim), dt, nsteps))
        self._keep[slot] = (workspace, u)

    def advance(self, stream=None) -> int:
        running = C.c_int32()
        A.check(self.lib.isdc_batch_advance(self._h, _stream_handle(stream), C.byref(running)))
        return running.value

    def time_sweeps(self, reps: int, graph: bool, stream) -> tuple:
        """(microseconds per sweep, launches per sweep) of `reps` extra sweeps
        of the running slots, eager or replayed from a captured HIP graph
        (isdc_batch_time_sweeps); the slots' states are left unspecified."""
        us, n = C.c_double(), C.c_int32()
        A.check(self.lib.isdc_batch_time_sweeps(self._h, reps, 1 if graph else 0, _stream_handle(stream),
                                                C.byref(us), C.byref(n)))
        return us.value, n.value

    def info(self, slot: int):
        state, status, steps = C.c_int32(), C.c_int32(), C.c_int32()
        st = A.Stats()
        A.check(self.lib.isdc_batch_slot_info(self._h, slot, C.byref(state), C.byref(status), C.byref(steps),
                                              C.byref(st)))
        return state.value, A.STATUS_NAMES.get(status.value, status.value), steps.value, StepStats.from_c(st, status.value)

    def release(self, slot: int):
        A.check(self.lib.isdc_batch_release(self._h, slot))
        self._keep[slot] = None

    def run(self, stream=None, max_advances: int = 1_000_000) -> int:
        """Advance until no slot is running; returns the number of batch sweeps."""
        k = 0
        while self.advance(stream) > 0:
            k += 1
            if k >= max_advances:
                raise RuntimeError("batch did not finish")
        return k + 1


class FixedBatch:
    """`count` fixed instances stepped together (isdc_batch_create /
    isdc_batch_step): instance i is (dims, n_i, nu_i, f^E_i, params_i); one
    torch workspace holds the batch arrays and every instance's plan."""

    def __init__(self, dim: int, instances, device=None):
        """instances: list of dicts with keys n, nu, fe_kind (optional) and the
        isdc_params fields (node_kind, M, vcycles, precision, sdc_tol, ...)."""
        self.lib = A.load()
        self.dim = dim
        self.count = len(instances)
        probs = (A.Problem * self.count)()
        pars = (A.Params * self.count)()
        self.n = []
        for i, inst in enumerate(instances):
            inst = dict(inst)
            n = inst.pop("n")
            nu = inst.pop("nu")
            fe = inst.pop("fe_kind", A.FE_ZERO)
            probs[i] = make_problem(dim, n, nu, fe)
            pars[i] = make_params(**inst)
            self.n.append(n)
        self._probs, self._pars = probs, pars
        nbytes = C.c_size_t()
        A.check(self.lib.isdc_batch_bytes(self.count, probs, pars, C.byref(nbytes)))
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        A.check(self.lib.isdc_batch_create(self.count, probs, pars, C.c_void_p(self.workspace.data_ptr()),
                                           nbytes.value, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.isdc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, us, dts, active=None, stream=None):
        """One time step of every active instance in place on us[i] (float64,
        shape (n_i,)*dim) with step dts[i]; returns (status, [StepStats or None])."""
        if len(us) != self.count or len(dts) != self.count:
            raise ValueError(f"need {self.count} states and step sizes")
        ptrs = (C.c_void_p * self.count)()
        for i, u in enumerate(us):
            on = active is None or active[i]
            ptrs[i] = _dev_ptr(u, torch.float64, self.n[i] ** self.dim).value if on else None
        dt = (C.c_double * self.count)(*dts)
        flags = [1] * self.count if active is None else [1 if a else 0 for a in active]
        act = (C.c_int32 * self.count)(*flags)
        stats = (A.Stats * self.count)()
        rc = self.lib.isdc_batch_step(self._h, ptrs, dt, act, _stream_handle(stream), stats)
        A.check(rc, allow=(A.E_NOT_CONVERGED, A.E_DIVERGED))
        out = []
        for i in range(self.count):
            on = active is None or active[i]
            out.append(StepStats.from_c(stats[i], A.OK) if on else None)
        return A.STATUS_NAMES.get(rc, rc), out
