"""Geometric multigrid V-cycle for (I - c L_h) u = rhs, in float64 or float32.

Test infrastructure only (see the package docstring).

Paper basis: Sec. 3 solves the implicit system of eq. (4) with spatial
multigrid; classical SDC cycles until a tolerance is met, ISDC applies a fixed
small number L of V-cycles (Sec. 3; L = 2 in Sec. 4.1).  The paper does not
describe the multigrid components (the solver came from a collaborator, see
the acknowledgments), so this oracle fixes textbook ones:

* grids with n_l = 2^(k-l) - 1 interior points per axis, h_l = 2^l h;
* rediscretised coarse operators A_l = I - c L_{h_l};
* smoother: red-black Gauss-Seidel (red = even sum of 0-based indices, updated
  first) or weighted Jacobi with omega = 2d / (2d + 1);
* full-weighting restriction (1/4, 1/2, 1/4 per axis, tensor product) and
  (bi/tri)linear prolongation;
* exact solve on the single-point grid, where every neighbour is a boundary
  ghost: u = rhs / (1 + 2 d c / h_l^2).

All arithmetic stays in the dtype of the arrays passed in (float32 arrays give
the float32 V-cycle of the mixed-precision path).
"""

from __future__ import annotations

import numpy as np

from .operators import apply_shifted, laplacian

SMOOTH_RBGS = 0
SMOOTH_JACOBI = 1


def level_sizes(n: int) -> list[int]:
    """Interior points per axis on every level, finest first: n, (n-1)/2, ..., 1."""
    if n < 1 or (n + 1) & n:
        raise ValueError("n must be 2^k - 1")
    sizes = [n]
    while sizes[-1] > 1:
        sizes.append((sizes[-1] - 1) // 2)
    return sizes


def _neighbour_sum(u: np.ndarray) -> np.ndarray:
    p = np.pad(u, 1)
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        lo = [slice(1, -1)] * u.ndim
        hi = [slice(1, -1)] * u.ndim
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        out += p[tuple(lo)] + p[tuple(hi)]
    return out


def _colour_mask(shape) -> np.ndarray:
    idx = np.indices(shape).sum(axis=0)
    return (idx % 2) == 0  # True = red


def smooth(u: np.ndarray, rhs: np.ndarray, c: float, h: float, kind: int,
           omega: float | None = None) -> np.ndarray:
    """One smoothing step on (I - c L_h) u = rhs; returns the new iterate.

    Weighted Jacobi: u + omega (rhs - A u) / D with D = 1 + 2 d c / h^2.
    Red-black Gauss-Seidel: all red points from the black ones, then all black
    points from the new red ones (each colour's neighbours have the other
    colour, so updating a whole colour at once is the sequential sweep).
    """
    t = u.dtype.type
    d = u.ndim
    a = t(c / (h * h))
    D = t(1.0) + t(2 * d) * a
    if kind == SMOOTH_JACOBI:
        w = t(omega if omega is not None else 2.0 * d / (2.0 * d + 1.0))
        return u + w * (rhs - apply_shifted(u, c, h)) / D
    if kind == SMOOTH_RBGS:
        red = _colour_mask(u.shape)
        v = u.copy()
        for mask in (red, ~red):
            new = (rhs + a * _neighbour_sum(v)) / D
            v[mask] = new[mask]
        return v
    raise ValueError(f"unknown smoother {kind}")


def _fw_axis(r: np.ndarray, ax: int) -> np.ndarray:
    n = r.shape[ax]
    nc = (n - 1) // 2
    take = lambda start: np.take(r, np.arange(start, start + 2 * nc, 2), axis=ax)  # noqa: E731
    q, hf = r.dtype.type(0.25), r.dtype.type(0.5)
    return q * take(0) + hf * take(1) + q * take(2)


def restrict_fw(r: np.ndarray) -> np.ndarray:
    """Full weighting: r_c[I] = r[2I]/4 + r[2I+1]/2 + r[2I+2]/4 on every axis."""
    for ax in range(r.ndim):
        r = _fw_axis(r, ax)
    return r


def _lin_axis(ec: np.ndarray, ax: int) -> np.ndarray:
    nc = ec.shape[ax]
    shape = list(ec.shape)
    shape[ax] = 2 * nc + 1
    out = np.zeros(shape, dtype=ec.dtype)
    pad = [(0, 0)] * ec.ndim
    pad[ax] = (1, 1)
    p = np.pad(ec, pad)  # e_c[-1] = e_c[nc] = 0
    odd = [slice(None)] * ec.ndim
    odd[ax] = slice(1, None, 2)
    even = [slice(None)] * ec.ndim
    even[ax] = slice(0, None, 2)
    left = [slice(None)] * ec.ndim
    left[ax] = slice(0, nc + 1)
    right = [slice(None)] * ec.ndim
    right[ax] = slice(1, nc + 2)
    out[tuple(odd)] = ec
    out[tuple(even)] = ec.dtype.type(0.5) * (p[tuple(left)] + p[tuple(right)])
    return out


def prolong_linear(ec: np.ndarray) -> np.ndarray:
    """Linear interpolation: e[2I+1] = e_c[I], e[2I] = (e_c[I-1] + e_c[I]) / 2."""
    for ax in range(ec.ndim):
        ec = _lin_axis(ec, ax)
    return ec


def vcycle(u: np.ndarray, rhs: np.ndarray, c: float, h: float,
           smoother: int = SMOOTH_RBGS, nu1: int = 1, nu2: int = 1,
           omega: float | None = None) -> np.ndarray:
    """One V(nu1, nu2)-cycle for (I - c L_h) u = rhs starting from ``u``."""
    t = u.dtype.type
    n = u.shape[0]
    d = u.ndim
    if n == 1:
        return rhs / (t(1.0) + t(2 * d) * t(c / (h * h)))
    for _ in range(nu1):
        u = smooth(u, rhs, c, h, smoother, omega)
    r = rhs - apply_shifted(u, c, h)
    rc = restrict_fw(r)
    ec = vcycle(np.zeros_like(rc), rc, c, 2.0 * h, smoother, nu1, nu2, omega)
    u = u + prolong_linear(ec)
    for _ in range(nu2):
        u = smooth(u, rhs, c, h, smoother, omega)
    return u


def residual_inf(u: np.ndarray, rhs: np.ndarray, c: float, h: float) -> float:
    """max |rhs - (I - c L_h) u| (in the dtype of the arrays)."""
    return float(np.max(np.abs(rhs - apply_shifted(u, c, h))))


__all__ = ["SMOOTH_RBGS", "SMOOTH_JACOBI", "level_sizes", "smooth", "restrict_fw",
           "prolong_linear", "vcycle", "residual_inf", "laplacian"]
