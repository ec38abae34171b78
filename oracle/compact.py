"""Fourth-order compact Laplacian with weighting matrix W (Sec. 3, eq. (5)).

Test infrastructure only (see the package docstring).

Paper basis: Sec. 3 discretises the Laplacian with a high-order compact
finite-difference stencil; the scheme carries a weighting matrix W on the
right-hand side, so that with f~^I = W f^I the semi-implicit sweep becomes
eq. (5), whose implicit operator is W - dt_m A, and the SDC residual needs W
inverted once per node.  The paper cites the stencil but does not print it.
This oracle takes the classical fourth-order compact ("Mehrstellen") scheme on
the interior points of [0, 1]^d with homogeneous Dirichlet boundary:

    A_h = L_h + (h^2 / 6) sum_{i<j} D_i D_j
    W   = I + (h^2 / 12) L_h

with L_h the second-order Laplacian and D_i the second difference along axis i
divided by h^2 (1D: the 3-point stencil and W = (1, 10, 1) / 12; 2D: the
9-point stencil (4 sum of edge neighbours + sum of corners - 20 centre) /
(6 h^2) and W = (8 centre + 4 neighbours) / 12; 3D: the 19-point stencil and
W = (6 centre + 6 neighbours) / 12).  W^{-1} A_h approximates the Laplacian to
O(h^4).  Both are diagonal in the sine basis:

    lambda_A = sum_i mu_i + (h^2 / 6) sum_{i<j} mu_i mu_j,
    lambda_W = 1 + (h^2 / 12) sum_i mu_i,     mu_i = -(4 / h^2) sin^2(a_i pi h / 2).

In eq. (5) the paper's A (the discretised f^I) is nu A_h here.

Multigrid for B = W - c A_h (c = dt_m nu), the operator of eq. (5).  The
paper does not describe its solver; this oracle rediscretises the continuous
operator behind B on every level: B_H = I + w L_H - c A_H with w = h^2 / 12
fixed by the finest grid (on the finest level B_h = W - c A_h exactly), and
uses weighted-Jacobi smoothing (red-black ordering is not a Gauss-Seidel sweep
for a 9-point stencil), full weighting, linear interpolation and an exact
solve on the one-point grid.  W itself (the residual's inversion) is the
5-point operator I - (-w) L_H, the form the second-order multigrid already
solves with a negative coefficient.
"""

from __future__ import annotations

import numpy as np

from .multigrid import restrict_fw, prolong_linear
from .operators import laplacian, laplacian_eigenvalues


def _second_difference(u: np.ndarray, ax: int) -> np.ndarray:
    """u[i-1] - 2 u[i] + u[i+1] along axis ax, zero ghosts (not divided by h^2)."""
    p = np.pad(u, 1)
    lo = [slice(1, -1)] * u.ndim
    hi = [slice(1, -1)] * u.ndim
    lo[ax] = slice(0, -2)
    hi[ax] = slice(2, None)
    return p[tuple(lo)] - u.dtype.type(2) * u + p[tuple(hi)]


def laplacian_compact(u: np.ndarray, h: float) -> np.ndarray:
    """A_h u = L_h u + (h^2/6) sum_{i<j} D_i D_j u (zero ghosts; keeps the dtype)."""
    t = u.dtype.type
    out = laplacian(u, h)
    for i in range(u.ndim):
        di = _second_difference(u, i)
        for j in range(i + 1, u.ndim):
            out = out + t(1.0 / (6.0 * h * h)) * _second_difference(di, j)
    return out


def weight(u: np.ndarray, h: float, w: float | None = None) -> np.ndarray:
    """W u = u + w L_h u with w = h^2/12 unless given (keeps the dtype)."""
    w = h * h / 12.0 if w is None else w
    return u + u.dtype.type(w) * laplacian(u, h)


def compact_eigenvalues(n: int, d: int, h: float):
    """(lambda_A, lambda_W) of the sine modes, shape (n,)*d, indexed by a_i - 1."""
    a = np.arange(1, n + 1)
    mu1 = -(4.0 / (h * h)) * np.sin(a * np.pi * h / 2.0) ** 2
    mus = []
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        mus.append(mu1.reshape(shape))
    lam_l = laplacian_eigenvalues(n, d, h)
    lam_a = lam_l.copy()
    for i in range(d):
        for j in range(i + 1, d):
            lam_a = lam_a + (h * h / 6.0) * mus[i] * mus[j]
    lam_w = 1.0 + (h * h / 12.0) * lam_l
    return lam_a, lam_w


def solve_weight_exact(y: np.ndarray, h: float) -> np.ndarray:
    """W^{-1} y by type-I discrete sine transform (the residual's inversion, Sec. 3)."""
    from scipy.fft import dstn, idstn

    _, lam_w = compact_eigenvalues(y.shape[0], y.ndim, h)
    return idstn(dstn(y, type=1, norm="ortho") / lam_w, type=1, norm="ortho")


def apply_compact_shifted(u: np.ndarray, c: float, h: float, w: float | None = None) -> np.ndarray:
    """B u = u + w L_h u - c A_h u; with the default w = h^2/12 this is (W - c A_h) u."""
    return weight(u, h, w) - u.dtype.type(c) * laplacian_compact(u, h)


def solve_compact_shifted_exact(rhs: np.ndarray, c: float, h: float) -> np.ndarray:
    """(W - c A_h)^{-1} rhs by sine transform: the full solve of classical SDC."""
    from scipy.fft import dstn, idstn

    lam_a, lam_w = compact_eigenvalues(rhs.shape[0], rhs.ndim, h)
    return idstn(dstn(rhs, type=1, norm="ortho") / (lam_w - c * lam_a), type=1, norm="ortho")


def compact_diagonal(d: int, c: float, w: float, H: float) -> float:
    """Centre coefficient of B_H = I + w L_H - c A_H.

    The centre of L_H is -2d/H^2; A_H adds 4/(6 H^2) for each of its
    d(d-1)/2 mixed differences D_i D_j."""
    pairs = d * (d - 1) // 2
    centre_a = (-2.0 * d + 4.0 * pairs / 6.0) / (H * H)
    return 1.0 + w * (-2.0 * d) / (H * H) - c * centre_a


def smooth_compact(u: np.ndarray, rhs: np.ndarray, c: float, w: float, H: float, omega: float) -> np.ndarray:
    """One weighted-Jacobi step on B_H u = rhs: u + omega (rhs - B_H u) / b0."""
    t = u.dtype.type
    b0 = t(compact_diagonal(u.ndim, c, w, H))
    return u + t(omega) * (rhs - apply_compact_shifted(u, c, H, w)) / b0


def vcycle_compact(u: np.ndarray, rhs: np.ndarray, c: float, h: float, nu1: int = 2, nu2: int = 2,
                   omega: float = 1.0, w: float | None = None) -> np.ndarray:
    """One V-cycle for B_H u = rhs on the level with spacing h (w fixed by the finest grid)."""
    w = h * h / 12.0 if w is None else w
    n = u.shape[0]
    if n == 1:
        return (rhs / u.dtype.type(compact_diagonal(u.ndim, c, w, h))).astype(u.dtype)
    for _ in range(nu1):
        u = smooth_compact(u, rhs, c, w, h, omega)
    r = rhs - apply_compact_shifted(u, c, h, w)
    rc = restrict_fw(r)
    ec = vcycle_compact(np.zeros_like(rc), rc, c, 2.0 * h, nu1, nu2, omega, w)
    u = u + prolong_linear(ec)
    for _ in range(nu2):
        u = smooth_compact(u, rhs, c, w, h, omega)
    return u


def residual_compact_inf(u: np.ndarray, rhs: np.ndarray, c: float, h: float) -> float:
    """max |rhs - (W - c A_h) u| (the inner residual of the compact solve)."""
    return float(np.max(np.abs(rhs - apply_compact_shifted(u, c, h))))
