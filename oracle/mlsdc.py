"""Two-level MLSDC with ISDC sweeps: SDC sweeps on a fine and a spatially
coarsened level, connected by an FAS correction (Sec. 5).

Test infrastructure only (see the package docstring).

Paper basis: Sec. 5 names the multi-level form of SDC as the natural place
for ISDC sweeps: sweeps run in a multigrid-like way on several levels, the
coarser levels use a coarser spatial representation of the problem, and the
levels are tied together by an FAS correction term; ISDC's L V-cycles are
its "reduced implicit solve".  The paper does not print the algorithm; this
oracle takes the standard two-level iteration:

1. one sweep of eq. (4) on the fine level (n points per axis, spacing h);
2. restriction of the node values to the coarse level (n_c = (n-1)/2 points,
   spacing 2h) by injection, u_c[I] = u[2I+1] per axis, and of u_0;
3. the FAS term per node m = 1..M
       tau_m = R(dt sum_j q_{m,j} f_h(U_j)) - dt sum_j q_{m,j} f_2h(R U_j),
   which makes R U a solution of the coarse collocation problem
   U_c = R u_0 + dt Q F_2h(U_c) + tau whenever U solves the fine one;
4. one sweep on the coarse level from R U with the FAS term (same nodes, same
   sweep, same number of V-cycles per solve, on the rediscretised operator);
5. the coarse correction interpolated back, U_m += P(U_c,m - R U_m), with P
   fourth-order (cubic) Lagrange interpolation per axis through the coarse
   points and the zero boundary values (``prolong_cubic``): with the linear
   interpolation of the multigrid the iteration converges two to three times
   more slowly than plain SDC on the heat problems tried, the interpolation
   error of each correction being left to the next fine sweep;
6. the SDC residual of the fine level (Sec. 3) decides whether to stop.

The step's result is the fine level's (the last node, or the end-point
quadrature for Gauss-Legendre).  With ``coarsen=False`` both levels share the
fine grid and R = P = I, so the FAS term vanishes and one iteration is two
plain sweeps: a check of the FAS bookkeeping.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .sdc import SDCConfig, SDCState, SDCStats, sdc_begin, sdc_sweep, sdc_residual, sdc_result, _f


def inject(u: np.ndarray) -> np.ndarray:
    """Coarse value at coarse point I = fine value at fine point 2I+1, per axis."""
    return u[(slice(1, None, 2),) * u.ndim].copy()


def prolong_cubic(ec: np.ndarray) -> np.ndarray:
    """Cubic interpolation from the coarse points (fine 2I+1) to all fine
    points, one axis after the other.  Per axis the known values sit at fine
    positions -1 (boundary, 0), 1, 3, ..., n-2 (coarse values) and n
    (boundary, 0); an even fine point 2I takes the Lagrange cubic through the
    four known points around it (shifted inwards next to the boundary; a
    level with one coarse point uses the three points it has)."""
    out = ec
    for ax in range(ec.ndim):
        o = np.moveaxis(out, ax, 0)
        nc = o.shape[0]
        n = 2 * nc + 1
        zero = np.zeros((1,) + o.shape[1:])
        known = np.concatenate([zero, o, zero])        # values at positions -1, 1, ..., n
        pos = np.arange(-1, n + 1, 2, dtype=np.float64)
        fine = np.zeros((n,) + o.shape[1:])
        fine[1::2] = o
        for I in range(nc + 1):
            x = 2.0 * I
            st = min(max(I - 1, 0), nc + 2 - 4) if nc >= 2 else 0
            k = min(4, nc + 2)
            acc = np.zeros(o.shape[1:])
            for a in range(st, st + k):
                w = 1.0
                for b in range(st, st + k):
                    if b != a:
                        w *= (x - pos[b]) / (pos[a] - pos[b])
                acc = acc + w * known[a]
            fine[2 * I] = acc
        out = np.moveaxis(fine, 0, ax)
    return out


@dataclass
class MLSDCStats:
    iterations: int = 0
    vcycles: int = 0             # fine-level V-cycles
    coarse_vcycles: int = 0
    residual: float = float("inf")
    residual_hist: list = field(default_factory=list)
    status: str = "ok"


def _coarse_state(fine: SDCState, coarsen: bool):
    cfg = fine.cfg
    R = inject if coarsen else (lambda v: v.copy())
    hc = 2.0 * fine.h if coarsen else fine.h
    u0c = R(fine.u0)
    Uc = [u0c] + [R(fine.U[m]) for m in range(1, cfg.M + 1)]
    Fc = [_f(u, cfg, hc) for u in Uc]
    st = SDCState(u0=u0c, U=Uc, F=Fc, dt=fine.dt, h=hc, cfg=cfg, tau=fine.tau, Q=fine.Q, S=fine.S,
                  stats=SDCStats())
    return st, R


def fas_term(fine: SDCState, coarse: SDCState, R) -> list:
    """tau_m = R(dt Q_m F_h(U)) - dt Q_m F_2h(R U), m = 1..M (index 0 unused)."""
    M, dt = fine.cfg.M, fine.dt
    out = [None]
    for m in range(1, M + 1):
        qf = np.zeros_like(fine.u0)
        qc = np.zeros_like(coarse.u0)
        for j in range(1, M + 1):
            qf = qf + fine.Q[m - 1, j - 1] * fine.F[j]
            qc = qc + fine.Q[m - 1, j - 1] * coarse.F[j]
        out.append(R(dt * qf) - dt * qc)
    return out


def mlsdc_iteration(fine: SDCState, stats: MLSDCStats, coarsen: bool = True) -> float:
    """One two-level iteration (steps 1-6 of the module docstring); returns the fine residual."""
    cfg = fine.cfg
    v0 = fine.stats.vcycles
    sdc_sweep(fine)
    stats.vcycles += fine.stats.vcycles - v0
    coarse, R = _coarse_state(fine, coarsen)
    RU = [u.copy() for u in coarse.U]
    tau = fas_term(fine, coarse, R)
    sdc_sweep(coarse, fas=tau)  # its own residual (without tau) is not used
    stats.coarse_vcycles += coarse.stats.vcycles
    for m in range(1, cfg.M + 1):
        corr = coarse.U[m] - RU[m]
        fine.U[m] = fine.U[m] + (prolong_cubic(corr) if coarsen else corr)
        fine.F[m] = _f(fine.U[m], cfg, fine.h)
    res = sdc_residual(fine)
    stats.iterations += 1
    stats.residual = res
    stats.residual_hist.append(res)
    return res


def mlsdc_step(u0: np.ndarray, dt: float, h: float, cfg: SDCConfig, coarsen: bool = True,
               fixed_iterations: int | None = None):
    """One time step of two-level MLSDC: iterations until the fine SDC residual
    is below cfg.tol (at most cfg.max_sweeps).  Returns (u_{n+1}, stats)."""
    if coarsen and (u0.shape[0] < 3 or u0.shape[0] % 2 == 0):
        raise ValueError("coarsening needs n = 2^k - 1 >= 3 points per axis")
    fine = sdc_begin(u0, dt, h, cfg)
    stats = MLSDCStats()
    nmax = fixed_iterations if fixed_iterations is not None else cfg.max_sweeps
    for _ in range(nmax):
        res = mlsdc_iteration(fine, stats, coarsen)
        if not np.isfinite(res):
            stats.status = "diverged"
            break
        if fixed_iterations is None and res < cfg.tol:
            break
    else:
        if fixed_iterations is None:
            stats.status = "not_converged"
    return sdc_result(fine), stats, fine
