"""Spatial operators: the f^I / f^E split and the implicit Euler system.

Test infrastructure only (see the package docstring).

Paper basis: Sec. 3 takes the linearly implicit case f^I(u) = A u with A a
discretisation of the Laplacian; eq. (4) treats f^I implicitly and f^E
explicitly.  Here A = nu * L_h, the second-order (2d+1)-point finite-difference
Laplacian on the interior points x_i = (i + 1) h, i = 0..n-1, of [0, 1]^d with
homogeneous Dirichlet boundary (ghost values zero) -- the paper's own runs used
a fourth-order compact stencil instead (Sec. 3, eq. (5)); with the
second-order stencil the weighting matrix W of eq. (5) is the identity and
eq. (5) is eq. (4).  f^E is zero (heat equation, Sec. 4.1) or the cubic
reaction term u - u^3.
"""

from __future__ import annotations

import numpy as np

FE_ZERO = 0
FE_CUBIC = 1


def laplacian(u: np.ndarray, h: float) -> np.ndarray:
    """L_h u: sum over axes of (u[i-1] - 2 u[i] + u[i+1]) / h^2, zero ghosts.

    Keeps the dtype of ``u`` (float32 stays float32).
    """
    dt = u.dtype.type
    out = np.zeros_like(u)
    p = np.pad(u, 1)
    inv_h2 = dt(1.0 / (h * h))
    for ax in range(u.ndim):
        lo = [slice(1, -1)] * u.ndim
        hi = [slice(1, -1)] * u.ndim
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        out += (p[tuple(lo)] - dt(2) * u + p[tuple(hi)])
    return out * inv_h2


def laplacian_matrix(n: int, d: int, h: float) -> np.ndarray:
    """Dense matrix of L_h on n^d interior points (row-major, last axis fastest)."""
    T = (np.diag(-2.0 * np.ones(n)) + np.diag(np.ones(n - 1), 1)
         + np.diag(np.ones(n - 1), -1)) / (h * h)
    I = np.eye(n)
    if d == 1:
        return T
    if d == 2:
        return np.kron(T, I) + np.kron(I, T)
    if d == 3:
        return (np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I)
                + np.kron(np.kron(I, I), T))
    raise ValueError("d must be 1, 2 or 3")


def laplacian_eigenvalues(n: int, d: int, h: float) -> np.ndarray:
    """Eigenvalues of L_h for the sine modes prod_i sin(a_i pi x_i), a_i = 1..n.

    lambda_a = -(4 / h^2) sum_i sin^2(a_i pi h / 2); returned with shape (n,)*d,
    indexed by a_i - 1 (the order of the type-I discrete sine transform).
    """
    a = np.arange(1, n + 1)
    l1 = -(4.0 / (h * h)) * np.sin(a * np.pi * h / 2.0) ** 2
    lam = np.zeros((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        lam = lam + l1.reshape(shape)
    return lam


def f_implicit(u: np.ndarray, nu: float, h: float) -> np.ndarray:
    """f^I(u) = nu L_h u (Sec. 3: the linearly implicit part)."""
    return u.dtype.type(nu) * laplacian(u, h)


def f_explicit(u: np.ndarray, fe_kind: int) -> np.ndarray:
    """f^E(u): zero for the heat equation, u - u^3 for reaction-diffusion."""
    if fe_kind == FE_ZERO:
        return np.zeros_like(u)
    if fe_kind == FE_CUBIC:
        return u - u * u * u
    raise ValueError(f"unknown f^E kind {fe_kind}")


def f_explicit_derivative(u: np.ndarray, fe_kind: int) -> np.ndarray:
    """Pointwise derivative of f^E (for Newton on the collocation system)."""
    if fe_kind == FE_ZERO:
        return np.zeros_like(u)
    if fe_kind == FE_CUBIC:
        return 1.0 - 3.0 * u * u
    raise ValueError(f"unknown f^E kind {fe_kind}")


def apply_shifted(u: np.ndarray, c: float, h: float) -> np.ndarray:
    """(I - c L_h) u, the implicit Euler operator of eq. (4) with c = dt_m nu."""
    return u - u.dtype.type(c) * laplacian(u, h)


def solve_shifted_exact(rhs: np.ndarray, c: float, h: float) -> np.ndarray:
    """Exact solution of (I - c L_h) u = rhs by type-I discrete sine transform.

    The sine modes diagonalise L_h, so each transformed coefficient is divided
    by 1 - c lambda_a.  This is the 'full solve' of classical SDC taken to
    machine precision (Sec. 3).
    """
    from scipy.fft import dstn, idstn

    lam = laplacian_eigenvalues(rhs.shape[0], rhs.ndim, h)
    return idstn(dstn(rhs, type=1, norm="ortho") / (1.0 - c * lam), type=1, norm="ortho")
