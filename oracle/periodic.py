"""Periodic grids, the periodic compact stencil and WENO5 advection for viscous Burgers.

Test infrastructure only (see the package docstring).

Paper basis: Sec. 4.1's second test problem is the viscous Burgers equation
u_t + u u_x + u u_y = nu Lap(u) on [-1, 1]^2 with periodic boundaries,
u(x, 0) = exp(-|x|^2 / sigma^2), sigma = 0.1, treated IMEX: the Laplacian
(fourth-order compact stencil with weighting matrix W, Sec. 3) implicitly and
the advection term, discretised by a fifth-order WENO scheme, explicitly.
The paper names the scheme without printing it.  This oracle takes:

* n points per axis on [-1, 1), x_i = -1 + i h, h = 2 / n (n = 2^k); the
  printed diffusive CFL numbers nu dt / h^2 = 0.41, 4.1, 41 for dt = 1e-3
  fix h = 1/64, i.e. n = 128.
* The compact stencil of ``compact`` with periodic wrap-around:
  A_h = L_h + (h^2/6) sum_{i<j} D_i D_j, W = I + (h^2/12) L_h, both diagonal
  in the discrete Fourier basis with mu_k = -(4/h^2) sin^2(pi k / n).
* f^E(u) = -(d/dx + d/dy)(u^2 / 2) in conservation form: per axis the flux
  difference (F_{i+1/2} - F_{i-1/2}) / h, where F_{i+1/2} is the WENO5
  reconstruction of Jiang and Shu (three third-order candidate stencils,
  smoothness indicators, linear weights 1/10, 6/10, 3/10, epsilon = 1e-6)
  applied to the split fluxes f^(+/-) = (u^2/2 +/- alpha u) / 2 with the local
  Lax-Friedrichs speed alpha = max(|u_i|, |u_{i+1}|) of the interface:
  f^+ from the left-biased points i-2..i+2, f^- mirrored from i-1..i+3.
* Multigrid on periodic grids: coarse point I sits on fine point 2I (n -> n/2),
  full weighting r_c[I] = r[2I-1]/4 + r[2I]/2 + r[2I+1]/4 and linear
  interpolation e[2I] = e_c[I], e[2I+1] = (e_c[I] + e_c[I+1]) / 2 per axis
  (wrapped); B_H = I + w L_H - c A_H as in ``compact``, weighted Jacobi; on the
  one-point grid every neighbour is the point itself, B_H = I and u = rhs.
"""

from __future__ import annotations

import numpy as np

WENO_EPS = 1e-6


def grid_p(n: int):
    """(x, h) of the periodic grid with n points on [-1, 1)."""
    h = 2.0 / n
    return -1.0 + h * np.arange(n), h


def _shift(u, ax, s):
    """u at index i + s along axis ax (periodic)."""
    return np.roll(u, -s, axis=ax)


def _second_difference_p(u, ax):
    return _shift(u, ax, -1) - u.dtype.type(2) * u + _shift(u, ax, 1)


def laplacian_p(u: np.ndarray, h: float) -> np.ndarray:
    t = u.dtype.type
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        out += _second_difference_p(u, ax)
    return out * t(1.0 / (h * h))


def laplacian_compact_p(u: np.ndarray, h: float) -> np.ndarray:
    t = u.dtype.type
    out = laplacian_p(u, h)
    for i in range(u.ndim):
        di = _second_difference_p(u, i)
        for j in range(i + 1, u.ndim):
            out = out + t(1.0 / (6.0 * h * h)) * _second_difference_p(di, j)
    return out


def weight_p(u: np.ndarray, h: float, w: float | None = None) -> np.ndarray:
    w = h * h / 12.0 if w is None else w
    return u + u.dtype.type(w) * laplacian_p(u, h)


def apply_compact_shifted_p(u: np.ndarray, c: float, h: float, w: float | None = None) -> np.ndarray:
    """B u = u + w L_h u - c A_h u (periodic); default w = h^2/12 gives (W - c A_h) u."""
    return weight_p(u, h, w) - u.dtype.type(c) * laplacian_compact_p(u, h)


def eigenvalues_p(n: int, d: int, h: float):
    """(lambda_L, lambda_A, lambda_W) of the Fourier modes (FFT order), shape (n,)*d."""
    k = np.arange(n)
    mu1 = -(4.0 / (h * h)) * np.sin(np.pi * k / n) ** 2
    mus = []
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        mus.append(mu1.reshape(shape))
    lam_l = sum(mus) * np.ones((n,) * d)
    lam_a = lam_l.copy()
    for i in range(d):
        for j in range(i + 1, d):
            lam_a = lam_a + (h * h / 6.0) * mus[i] * mus[j]
    lam_w = 1.0 + (h * h / 12.0) * lam_l
    return lam_l, lam_a, lam_w


def solve_weight_exact_p(y: np.ndarray, h: float) -> np.ndarray:
    """W^{-1} y by the discrete Fourier transform."""
    _, _, lam_w = eigenvalues_p(y.shape[0], y.ndim, h)
    return np.real(np.fft.ifftn(np.fft.fftn(y) / lam_w))


def solve_compact_shifted_exact_p(rhs: np.ndarray, c: float, h: float) -> np.ndarray:
    """(W - c A_h)^{-1} rhs by the discrete Fourier transform."""
    _, lam_a, lam_w = eigenvalues_p(rhs.shape[0], rhs.ndim, h)
    return np.real(np.fft.ifftn(np.fft.fftn(rhs) / (lam_w - c * lam_a)))


def restrict_fw_p(r: np.ndarray) -> np.ndarray:
    """Full weighting onto the even points, per axis (periodic)."""
    t = r.dtype.type
    out = r
    for ax in range(r.ndim):
        full = t(0.25) * _shift(out, ax, -1) + t(0.5) * out + t(0.25) * _shift(out, ax, 1)
        idx = [slice(None)] * r.ndim
        idx[ax] = slice(0, None, 2)
        out = full[tuple(idx)]
    return out


def prolong_linear_p(ec: np.ndarray) -> np.ndarray:
    """Linear interpolation from the even points, per axis (periodic)."""
    t = ec.dtype.type
    out = ec
    for ax in range(ec.ndim):
        nc = out.shape[ax]
        shape = list(out.shape)
        shape[ax] = 2 * nc
        fine = np.zeros(shape, dtype=ec.dtype)
        ev = [slice(None)] * ec.ndim
        od = [slice(None)] * ec.ndim
        ev[ax] = slice(0, None, 2)
        od[ax] = slice(1, None, 2)
        fine[tuple(ev)] = out
        fine[tuple(od)] = t(0.5) * (out + _shift(out, ax, 1))
        out = fine
    return out


def compact_diagonal_p(d: int, c: float, w: float, H: float) -> float:
    """Centre coefficient of B_H on a periodic grid of at least two points per axis."""
    pairs = d * (d - 1) // 2
    centre_a = (-2.0 * d + 4.0 * pairs / 6.0) / (H * H)
    return 1.0 + w * (-2.0 * d) / (H * H) - c * centre_a


def vcycle_compact_p(u: np.ndarray, rhs: np.ndarray, c: float, h: float, nu1: int = 3, nu2: int = 3,
                     omega: float = 1.0, w: float | None = None) -> np.ndarray:
    """One weighted-Jacobi V-cycle for B_H u = rhs on a periodic level of spacing h."""
    w = h * h / 12.0 if w is None else w
    n = u.shape[0]
    if n == 1:
        return rhs.copy()  # every neighbour is the point itself: B_H = I
    t = u.dtype.type
    b0 = t(compact_diagonal_p(u.ndim, c, w, h))
    for _ in range(nu1):
        u = u + t(omega) * (rhs - apply_compact_shifted_p(u, c, h, w)) / b0
    rc = restrict_fw_p(rhs - apply_compact_shifted_p(u, c, h, w))
    ec = vcycle_compact_p(np.zeros_like(rc), rc, c, 2.0 * h, nu1, nu2, omega, w)
    u = u + prolong_linear_p(ec)
    for _ in range(nu2):
        u = u + t(omega) * (rhs - apply_compact_shifted_p(u, c, h, w)) / b0
    return u


def residual_compact_inf_p(u: np.ndarray, rhs: np.ndarray, c: float, h: float) -> float:
    return float(np.max(np.abs(rhs - apply_compact_shifted_p(u, c, h))))


def _weno5_left(a, b, c, d, e, eps=WENO_EPS):
    """WENO5 value at the right face of the middle point c from values a..e (left-biased)."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    a0 = 0.1 / (eps + b0) ** 2
    a1 = 0.6 / (eps + b1) ** 2
    a2 = 0.3 / (eps + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def weno5_flux(u: np.ndarray, ax: int, eps: float = WENO_EPS) -> np.ndarray:
    """Numerical flux F_{i+1/2} of u^2/2 along axis ax at every interface i+1/2 (periodic)."""
    s = lambda k: _shift(u, ax, k)  # noqa: E731  u_{i+k}
    alpha = np.maximum(np.abs(s(0)), np.abs(s(1)))
    fp = lambda k: 0.5 * (0.5 * s(k) * s(k) + alpha * s(k))  # noqa: E731  f^+ at i+k, interface speed
    fm = lambda k: 0.5 * (0.5 * s(k) * s(k) - alpha * s(k))  # noqa: E731
    plus = _weno5_left(fp(-2), fp(-1), fp(0), fp(1), fp(2), eps)
    minus = _weno5_left(fm(3), fm(2), fm(1), fm(0), fm(-1), eps)
    return plus + minus


def burgers_advection(u: np.ndarray, h: float, eps: float = WENO_EPS) -> np.ndarray:
    """f^E(u) = -sum over axes of (F_{i+1/2} - F_{i-1/2}) / h (periodic WENO5)."""
    out = np.zeros_like(u)
    for ax in range(u.ndim):
        F = weno5_flux(u, ax, eps)
        out -= (F - _shift(F, ax, -1)) / h
    return out
