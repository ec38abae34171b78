"""Semi-implicit SDC / ISDC sweeps, the SDC residual and the time step.

Test infrastructure only (see the package docstring).

Paper basis:

* Sweep: eq. (4).  For m = 0..M-1 (tau_0 = 0, dt_m = dt (tau_{m+1} - tau_m)):
    u_{m+1}^{k+1} = u_m^{k+1} + dt_m [f^I(u_{m+1}^{k+1}) - f^I(u_{m+1}^k)]
                    + dt_m [f^E(u_m^{k+1}) - f^E(u_m^k)] + S_m^{m+1} F(u^k),
  i.e. (I - dt_m nu L_h) u_{m+1}^{k+1} = rhs with
    rhs = u_m^{k+1} + dt_m [f^E(u_m^{k+1}) - f^E(u_m^k)] - dt_m f^I(u_{m+1}^k)
          + S_m^{m+1} F(u^k).
  u_0^k = u_0 for every k (the left end of the step).
* Inner solve (Sec. 3): classical SDC solves each system fully (``exact``:
  sine-transform direct solve; ``mg`` with ``vcycles = 0``: V-cycles until the
  inner residual is at most ``inner_tol``); ISDC applies exactly L V-cycles
  (``mg`` with ``vcycles = L``), optionally stopping early once ``inner_tol``
  is met.  The initial guess is u_{m+1}^k (Sec. 4.3); the ablation of Sec. 4.3
  replaces it by zero or by u_m^{k+1}.
* Residual (Sec. 3): max over nodes m = 1..M and grid points of
  |u_0 + dt sum_j q_{m,j} f(u_j^k) - u_m^k|; sweeps run until it is below the
  tolerance.
* Initial iterate: u_j^0 = u_0 at every node (the paper is silent; with this
  choice sweep 1 is plain implicit / IMEX Euler).  At least one sweep is made.
* Result: u_{n+1} = u_M (tau_M = 1 for Gauss-Lobatto and right Gauss-Radau).
* Mixed precision: the inner V-cycles run in float32 on the correction
  equation (I - c L_h) e = rhs - (I - c L_h) g for the guess g, with the
  right-hand side rounded to float32 and u = g + e accumulated in float64.
  The fixed point of the sweep is unchanged because that right-hand side
  vanishes at the collocation solution.
* Periodic boundaries (``bc = BC_PERIODIC``, compact stencil only) and the
  WENO5 Burgers advection (``fe_kind = FE_BURGERS``) follow periodic.py.
* Compact stencil (``stencil = STENCIL_COMPACT4``, eq. (5)): f~(u) =
  W f^E(u) + nu A_h u is kept per node, the implicit system is
  (W - dt_m nu A_h) u_{m+1}^{k+1} = W u_m^{k+1} + dt_m W [f^E(u_m^{k+1}) -
  f^E(u_m^k)] - dt_m nu A_h u_{m+1}^k + S_m^{m+1} F~(u^k), and the residual is
  u_0 + W^{-1} (dt sum_j q_{m,j} f~(u_j)) - u_m (W and A_h in compact.py).
  Its multigrid is the weighted-Jacobi V-cycle of compact.py.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .collocation import qmatrix, smatrix, nodes, end_weights, ends_on_node, NODES_LOBATTO
from . import compact as _cd
from . import periodic as _cp
from .multigrid import SMOOTH_RBGS, vcycle, residual_inf
from .operators import FE_ZERO, f_explicit, f_implicit, apply_shifted, solve_shifted_exact

STENCIL_2ND = 0
STENCIL_COMPACT4 = 1

BC_DIRICHLET = 0
BC_PERIODIC = 1            # [-1, 1)^d, compact stencil only (the Burgers setup of Sec. 4.1)

FE_BURGERS = 2             # f^E = -(d/dx + d/dy)(u^2/2), WENO5 (periodic only)

GUESS_PREV_SWEEP = 0
GUESS_ZERO = 1
GUESS_PREV_NODE = 2

PREC_FP64 = 0
PREC_MIXED = 1


class NotConverged(RuntimeError):
    pass


class Diverged(RuntimeError):
    pass


@dataclass
class SDCConfig:
    nu: float = 1.0
    fe_kind: int = FE_ZERO
    node_kind: int = NODES_LOBATTO
    M: int = 3
    inner: str = "mg"            # "exact" (direct solve) or "mg"
    vcycles: int = 2             # L; 0 = classical: cycle until inner_tol
    inner_tol: float = 1e-10
    early_exit: bool = False
    tol: float = 1e-10
    max_sweeps: int = 100
    smoother: int = SMOOTH_RBGS
    nu1: int = 1
    nu2: int = 1
    omega: float | None = None
    precision: int = PREC_FP64
    guess: int = GUESS_PREV_SWEEP
    max_classical_cycles: int = 100
    stencil: int = STENCIL_2ND
    bc: int = BC_DIRICHLET


@dataclass
class SDCStats:
    sweeps: int = 0
    vcycles: int = 0
    residual: float = float("inf")
    residual_hist: list = field(default_factory=list)
    status: str = "ok"           # "ok" | "not_converged" | "diverged"
    # smallest |res / inner_tol - 1| over every inner stopping test made (classical
    # mode and early exit); it tells the tests when a V-cycle count was decided at
    # the edge of the inner tolerance, where another rounding order may decide otherwise
    inner_margin: float = float("inf")


@dataclass
class SDCState:
    u0: np.ndarray
    U: list                      # U[j] = u_j^k, j = 1..M (index 0 unused: u_0)
    F: list                      # F[j] = f(u_j^k)
    dt: float
    h: float
    cfg: SDCConfig
    tau: np.ndarray
    Q: np.ndarray
    S: np.ndarray
    stats: SDCStats


class _Compact:
    """The compact-stencil operators of the configured boundary condition."""

    def __init__(self, bc):
        if bc == BC_PERIODIC:
            self.weight, self.lap = _cp.weight_p, _cp.laplacian_compact_p
            self.solve_w, self.solve = _cp.solve_weight_exact_p, _cp.solve_compact_shifted_exact_p
            self.apply, self.vcycle, self.res = (_cp.apply_compact_shifted_p, _cp.vcycle_compact_p,
                                                 _cp.residual_compact_inf_p)
        else:
            self.weight, self.lap = _cd.weight, _cd.laplacian_compact
            self.solve_w, self.solve = _cd.solve_weight_exact, _cd.solve_compact_shifted_exact
            self.apply, self.vcycle, self.res = (_cd.apply_compact_shifted, _cd.vcycle_compact,
                                                 _cd.residual_compact_inf)


def _check(cfg):
    if cfg.bc == BC_PERIODIC and cfg.stencil != STENCIL_COMPACT4:
        raise ValueError("periodic boundaries are provided with the compact stencil only")
    if cfg.fe_kind == FE_BURGERS and cfg.bc != BC_PERIODIC:
        raise ValueError("the WENO5 Burgers advection needs periodic boundaries")


def _fe(u, cfg, h):
    """f^E(u): pointwise kinds, or the periodic WENO5 Burgers advection."""
    if cfg.fe_kind == FE_BURGERS:
        return _cp.burgers_advection(u, h)
    return f_explicit(u, cfg.fe_kind)


def _f(u, cfg, h):
    """f(u) = nu L_h u + f^E(u); for the compact stencil f~(u) = W f^E(u) + nu A_h u."""
    if cfg.stencil == STENCIL_COMPACT4:
        op = _Compact(cfg.bc)
        return op.weight(_fe(u, cfg, h), h) + cfg.nu * op.lap(u, h)
    return f_implicit(u, cfg.nu, h) + _fe(u, cfg, h)


def sdc_residual(state: SDCState) -> float:
    """Max-norm SDC residual of the current iterate (Sec. 3)."""
    cfg = state.cfg
    per_node = []
    for m in range(1, cfg.M + 1):
        quad = np.zeros_like(state.u0)
        for j in range(1, cfg.M + 1):
            quad = quad + state.Q[m - 1, j - 1] * state.F[j]
        if cfg.stencil == STENCIL_COMPACT4:  # the stored values are W f: invert W once per node
            r = state.u0 + _Compact(cfg.bc).solve_w(state.dt * quad, state.h) - state.U[m]
        else:
            r = state.u0 + state.dt * quad - state.U[m]
        per_node.append(np.max(np.abs(r)))
    return float(np.max(per_node))  # np.max propagates NaN


def sdc_begin(u0: np.ndarray, dt: float, h: float, cfg: SDCConfig) -> SDCState:
    """Spread u_0 to every node and evaluate f there (initial iterate k = 0)."""
    _check(cfg)
    u0 = np.asarray(u0, dtype=np.float64)
    f0 = _f(u0, cfg, h)
    M = cfg.M
    U = [u0.copy() for _ in range(M + 1)]
    F = [f0.copy() for _ in range(M + 1)]
    return SDCState(u0=u0, U=U, F=F, dt=dt, h=h, cfg=cfg,
                    tau=nodes(cfg.node_kind, M), Q=qmatrix(cfg.node_kind, M),
                    S=smatrix(cfg.node_kind, M), stats=SDCStats())


def _inner_solve(rhs, guess, c, h, cfg, stats=None):
    """Solve (I - c L_h) u = rhs (compact: (W - c A_h) u = rhs); returns (u, V-cycles)."""
    compact = cfg.stencil == STENCIL_COMPACT4
    op = _Compact(cfg.bc)
    if cfg.inner == "exact":
        return (op.solve(rhs, c, h) if compact else solve_shifted_exact(rhs, c, h)), 0
    apply_op = op.apply if compact else apply_shifted
    res_inf = op.res if compact else residual_inf

    def cycle(v, b):
        if compact:
            return op.vcycle(v, b, c, h, cfg.nu1, cfg.nu2, cfg.omega if cfg.omega is not None else 1.0)
        return vcycle(v, b, c, h, cfg.smoother, cfg.nu1, cfg.nu2, cfg.omega)

    if cfg.precision == PREC_FP64:
        u = guess.copy()

        def inner_res():
            return res_inf(u, rhs, c, h)
    else:
        r32 = (rhs - apply_op(guess, c, h)).astype(np.float32)
        e = np.zeros_like(r32)

        def inner_res():
            return res_inf(e, r32, c, h)

    classical = cfg.vcycles == 0
    limit = cfg.max_classical_cycles if classical else cfg.vcycles
    check = classical or cfg.early_exit
    ncyc = 0
    while ncyc < limit:
        if check:
            res = inner_res()
            if stats is not None and cfg.inner_tol > 0:
                stats.inner_margin = min(stats.inner_margin, abs(res / cfg.inner_tol - 1.0))
            if res <= cfg.inner_tol:
                break
        if cfg.precision == PREC_FP64:
            u = cycle(u, rhs)
        else:
            e = cycle(e, r32)
        ncyc += 1
    if cfg.precision == PREC_FP64:
        return u, ncyc
    return guess + e.astype(np.float64), ncyc


def sdc_sweep(state: SDCState, fas: list | None = None) -> float:
    """One sweep of eq. (4) over all substeps; returns the new SDC residual.

    ``fas`` (multi-level use, see mlsdc.py): per node m = 1..M (index 0
    unused) a term tau_m added to the collocation equations of this level,
    U_m = u_0 + dt sum_j q_{m,j} f(U_j) + tau_m; the node-to-node form of the
    sweep then carries tau_{m+1} - tau_m (tau_0 = 0) next to S_m^{m+1} F."""
    cfg = state.cfg
    dt, h, M = state.dt, state.h, cfg.M
    tau_ext = np.concatenate([[0.0], state.tau])
    # S_m^{m+1} F(u^k) for every substep, from the previous iterate
    SF = []
    for m in range(M):
        acc = np.zeros_like(state.u0)
        for j in range(1, M + 1):
            acc = acc + state.S[m, j - 1] * state.F[j]
        sf = dt * acc
        if fas is not None:
            sf = sf + fas[m + 1] - (fas[m] if m > 0 else 0.0)
        SF.append(sf)
    Uold = [u for u in state.U]
    Unew = [None] * (M + 1)
    Fnew = [None] * (M + 1)
    Unew[0] = state.u0
    Uold[0] = state.u0
    for m in range(M):
        dtm = dt * (tau_ext[m + 1] - tau_ext[m])
        um_new, um_old, up_old = Unew[m], Uold[m], Uold[m + 1]
        c = dtm * cfg.nu
        explicit = um_new + dtm * (_fe(um_new, cfg, h) - _fe(um_old, cfg, h))
        if cfg.stencil == STENCIL_COMPACT4:  # eq. (5)
            op = _Compact(cfg.bc)
            rhs = op.weight(explicit, h) - c * op.lap(up_old, h) + SF[m]
        else:  # eq. (4)
            rhs = explicit - dtm * f_implicit(up_old, cfg.nu, h) + SF[m]
        if dtm == 0.0:
            # degenerate substep (tau_1 = 0 for Gauss-Lobatto): the operator is I (or W)
            u = _Compact(cfg.bc).solve_w(rhs, h) if cfg.stencil == STENCIL_COMPACT4 else rhs
        else:
            if cfg.guess == GUESS_PREV_SWEEP:
                g = up_old
            elif cfg.guess == GUESS_ZERO:
                g = np.zeros_like(up_old)
            elif cfg.guess == GUESS_PREV_NODE:
                g = um_new
            else:
                raise ValueError("unknown guess mode")
            u, ncyc = _inner_solve(rhs, g, c, h, cfg, state.stats)
            state.stats.vcycles += ncyc
        Unew[m + 1] = u
        Fnew[m + 1] = _f(u, cfg, h)
    Fnew[0] = state.F[0]
    state.U = Unew
    state.F = Fnew
    state.stats.sweeps += 1
    res = sdc_residual(state)
    state.stats.residual = res
    state.stats.residual_hist.append(res)
    return res


def sdc_step(u0: np.ndarray, dt: float, h: float, cfg: SDCConfig,
             fixed_sweeps: int | None = None, raise_on_failure: bool = False):
    """One ISDC / SDC time step: sweeps until residual < tol (Sec. 3, Sec. 4.2).

    With ``fixed_sweeps`` set, exactly that many sweeps are made and no stopping
    test is applied.  Returns (u_{n+1}, stats).
    """
    st = sdc_begin(u0, dt, h, cfg)
    nmax = fixed_sweeps if fixed_sweeps is not None else cfg.max_sweeps
    for _ in range(nmax):
        res = sdc_sweep(st)
        if not np.isfinite(res):
            st.stats.status = "diverged"
            if raise_on_failure:
                raise Diverged(f"non-finite SDC residual after {st.stats.sweeps} sweeps")
            break
        if fixed_sweeps is None and res < cfg.tol:
            break
    else:
        if fixed_sweeps is None:
            st.stats.status = "not_converged"
            if raise_on_failure:
                raise NotConverged(f"residual {st.stats.residual:.3e} after {nmax} sweeps")
    return sdc_result(st), st.stats


def sdc_result(state: SDCState) -> np.ndarray:
    """u(T_{n+1}) of the current iterate: the last node value where tau_M = 1,
    else (Gauss-Legendre) the collocation polynomial at the end of the step,
    u_0 + dt sum_j b_j f_j (compact stencil: u_0 + W^{-1}(dt sum_j b_j f~_j))."""
    cfg = state.cfg
    if ends_on_node(cfg.node_kind):
        return state.U[cfg.M].copy()
    b = end_weights(cfg.node_kind, cfg.M)
    acc = np.zeros_like(state.u0)
    for j in range(1, cfg.M + 1):
        acc = acc + b[j - 1] * state.F[j]
    if cfg.stencil == STENCIL_COMPACT4:
        return state.u0 + _Compact(cfg.bc).solve_w(state.dt * acc, state.h)
    return state.u0 + state.dt * acc


def sdc_run(u0: np.ndarray, dt: float, h: float, cfg: SDCConfig, nsteps: int):
    """nsteps consecutive time steps; returns (u, list of per-step stats)."""
    u = np.asarray(u0, dtype=np.float64)
    all_stats = []
    for _ in range(nsteps):
        u, st = sdc_step(u, dt, h, cfg)
        all_stats.append(st)
        if st.status != "ok":
            break
    return u, all_stats
