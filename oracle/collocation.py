"""Collocation nodes, quadrature matrices and the direct collocation solution.

Test infrastructure only (see the package docstring).

Paper basis:

* The nodes are those of a spectral collocation rule (Gauss-Legendre,
  Gauss-Radau or Gauss-Lobatto; Sec. 1, and Sec. 2 right after eq. (2)).  This
  oracle provides Gauss-Lobatto, right Gauss-Radau and Gauss-Legendre.  The
  first two end on the right end point of the step, so u(T_{n+1}) is the last
  node value; Gauss-Legendre nodes are all interior, and the step's result is
  the collocation polynomial at the end point, u_0 + dt * sum_j b_j f(u_j) with
  b_j the integral of l_j over the whole step (``end_weights``).
* eq. (2): the node-to-node integral over [t_m, t_{m+1}] is approximated by
  dt * sum_j s_{m,j} f(u_j) = S_m^{m+1} F(u), with F(u) = (f(u_1), ..., f(u_M)).
* eq. (1) written at the nodes gives the collocation problem
  U_m = u_0 + dt * sum_j q_{m,j} f(U_j), m = 1..M, whose solution SDC iterates
  towards (Sec. 1: the large M*d-by-M*d system).

Conventions: nodes tau_1 < ... < tau_M lie in [0, 1] (unit step); tau_0 := 0 is
the left end of the step.  ``qmatrix`` returns Q with Q[m-1, j-1] = q_{m,j} =
integral over [0, tau_m] of the Lagrange polynomial l_j on tau_1..tau_M.
``smatrix`` returns S with S[m, j-1] = s_{m,j} = q_{m+1,j} - q_{m,j},
m = 0..M-1, q_{0,j} = 0.
"""

from __future__ import annotations

import mpmath as mp
import numpy as np
from numpy.polynomial import legendre as npleg

NODES_LOBATTO = 0
NODES_RADAU_RIGHT = 1
NODES_LEGENDRE = 2

_DPS = 40  # working precision (decimal digits) for node and weight polishing


def _polish(fun, x0):
    with mp.workdps(_DPS):
        return mp.findroot(fun, mp.mpf(float(x0)), tol=mp.mpf(10) ** (-(_DPS - 5)))


def _nodes_mp(kind: int, M: int):
    """Nodes on [-1, 1] as mpmath numbers (sorted ascending)."""
    with mp.workdps(_DPS):
        if kind == NODES_LOBATTO:
            if M < 2:
                raise ValueError("Gauss-Lobatto needs M >= 2")
            n = M - 1
            # interior Lobatto points: roots of P'_n.  Starting values from
            # numpy, refined on (1 - x^2) P'_n(x) / n = P_{n-1}(x) - x P_n(x).
            coef = np.zeros(n + 1)
            coef[n] = 1.0
            start = np.sort(np.real(npleg.legroots(npleg.legder(coef)))) if n >= 2 else []
            g = lambda x: mp.legendre(n - 1, x) - x * mp.legendre(n, x)  # noqa: E731
            inner = [_polish(g, x) for x in start]
            pts = [mp.mpf(-1)] + inner + [mp.mpf(1)]
        elif kind == NODES_RADAU_RIGHT:
            if M < 1:
                raise ValueError("Gauss-Radau needs M >= 1")
            # right Radau points: roots of P_M - P_{M-1} (x = +1 is one of them)
            coef = np.zeros(M + 1)
            coef[M] = 1.0
            coef[M - 1] -= 1.0
            start = np.sort(np.real(npleg.legroots(coef)))
            g = lambda x: mp.legendre(M, x) - mp.legendre(M - 1, x)  # noqa: E731
            pts = [_polish(g, x) for x in start[:-1]] + [mp.mpf(1)]
        elif kind == NODES_LEGENDRE:
            if M < 1:
                raise ValueError("Gauss-Legendre needs M >= 1")
            pts = _gauss_legendre_mp(M)[0]  # roots of P_M, all interior
        else:
            raise ValueError(f"unknown node kind {kind}")
        return sorted(pts)


def nodes(kind: int, M: int) -> np.ndarray:
    """Collocation nodes tau_1..tau_M on the unit step [0, 1] (float64).

    Sec. 1 and Sec. 2 (after eq. (2)): Gauss-Lobatto (both end points), right
    Gauss-Radau (right end point only) or Gauss-Legendre (no end point);
    tau = (1 + x) / 2 for x in [-1, 1].
    """
    with mp.workdps(_DPS):
        return np.array([float((1 + x) / 2) for x in _nodes_mp(kind, M)])


def _gauss_legendre_mp(npts: int):
    """Gauss-Legendre points and weights on [-1, 1] in mpmath precision."""
    with mp.workdps(_DPS):
        x0, _ = npleg.leggauss(npts)
        xs = [_polish(lambda x: mp.legendre(npts, x), x) for x in x0]
        ws = []
        for x in xs:
            # P'_n(x) = n (P_{n-1}(x) - x P_n(x)) / (1 - x^2); P_n(x) = 0 at a root
            dp = npts * mp.legendre(npts - 1, x) / (1 - x * x)
            ws.append(2 / ((1 - x * x) * dp * dp))
        return xs, ws


def _q_mp(kind: int, M: int):
    with mp.workdps(_DPS):
        tau = [(1 + x) / 2 for x in _nodes_mp(kind, M)]
        gx, gw = _gauss_legendre_mp(M + 1)  # exact for degree <= 2M+1 > M-1

        def lag(j, s):
            v = mp.mpf(1)
            for i in range(M):
                if i != j:
                    v *= (s - tau[i]) / (tau[j] - tau[i])
            return v

        Q = [[mp.mpf(0)] * M for _ in range(M)]
        for m in range(M):
            b = tau[m]  # integrate over [0, tau_m]
            for j in range(M):
                acc = mp.mpf(0)
                for x, w in zip(gx, gw):
                    acc += w * lag(j, b * (x + 1) / 2)
                Q[m][j] = acc * b / 2
        return tau, Q


def end_weights(kind: int, M: int) -> np.ndarray:
    """b_j = integral over the whole step [0, 1] of l_j (the collocation rule's
    quadrature weights); u(T_{n+1}) = u_0 + dt * sum_j b_j f(u_j).  For the node
    families that end on tau_M = 1 this is the last row of Q."""
    with mp.workdps(_DPS):
        tau = [(1 + x) / 2 for x in _nodes_mp(kind, M)]
        gx, gw = _gauss_legendre_mp(M + 1)
        out = []
        for j in range(M):
            acc = mp.mpf(0)
            for x, w in zip(gx, gw):
                s = (x + 1) / 2
                v = mp.mpf(1)
                for i in range(M):
                    if i != j:
                        v *= (s - tau[i]) / (tau[j] - tau[i])
                acc += w * v
            out.append(float(acc / 2))
        return np.array(out)


def ends_on_node(kind: int) -> bool:
    """True if tau_M = 1, so that the last node value is the step's result."""
    return kind in (NODES_LOBATTO, NODES_RADAU_RIGHT)


def qmatrix(kind: int, M: int) -> np.ndarray:
    """Cumulative collocation matrix, Q[m-1, j-1] = integral_0^{tau_m} l_j.

    Eq. (1) at the nodes (Sec. 2).  Each entry is the exact integral of a
    polynomial of degree M-1, computed with an (M+1)-point Gauss-Legendre rule
    on [0, tau_m] in 40-digit arithmetic.
    """
    _, Q = _q_mp(kind, M)
    return np.array([[float(v) for v in row] for row in Q])


def smatrix(kind: int, M: int) -> np.ndarray:
    """Node-to-node quadrature matrix of eq. (2): S[m] = Q[m] - Q[m-1], Q[-1] = 0.

    Row m (m = 0..M-1) integrates from tau_m to tau_{m+1} with tau_0 = 0; the
    entries are differenced in 40-digit arithmetic before rounding.
    """
    _, Q = _q_mp(kind, M)
    with mp.workdps(_DPS):
        rows = []
        for m in range(M):
            prev = Q[m - 1] if m > 0 else [mp.mpf(0)] * M
            rows.append([float(Q[m][j] - prev[j]) for j in range(M)])
    return np.array(rows)


def stability_function(z, kind: int, M: int):
    """Collocation stability function R(z) for u' = lambda u, z = dt * lambda.

    The collocation problem (Sec. 1) for a scalar linear ODE is the M-by-M
    system (I - z Q) U = u_0 * 1; R(z) = U_M / u_0 where tau_M = 1 (Lobatto,
    Radau), else R(z) = 1 + z * sum_j b_j U_j / u_0 (Gauss-Legendre).  ``z``
    may be a scalar or an array.
    """
    Q = qmatrix(kind, M)
    z = np.asarray(z, dtype=np.float64)
    flat = z.reshape(-1)
    A = np.eye(M)[None, :, :] - flat[:, None, None] * Q[None, :, :]
    U = np.linalg.solve(A, np.ones((flat.size, M, 1)))[:, :, 0]
    if ends_on_node(kind):
        return U[:, -1].reshape(z.shape)
    return (1.0 + flat * (U @ end_weights(kind, M))).reshape(z.shape)


def collocation_heat_modal(u0: np.ndarray, dt: float, nu: float, h: float,
                           kind: int, M: int) -> np.ndarray:
    """Direct collocation solution u(T_{n+1}) for the linear problem u' = nu L_h u.

    Sec. 1 (the coupled collocation system).  L_h has the discrete sine
    functions as eigenvectors, so the M*N-by-M*N system decouples into one
    M-by-M system per sine mode: each coefficient is multiplied by R(dt nu lambda_a).
    """
    from scipy.fft import dstn, idstn

    from .operators import laplacian_eigenvalues

    d = u0.ndim
    n = u0.shape[0]
    lam = laplacian_eigenvalues(n, d, h)
    coef = dstn(u0, type=1, norm="ortho")
    return idstn(coef * stability_function(dt * nu * lam, kind, M), type=1, norm="ortho")


def collocation_dense(u0: np.ndarray, dt: float, nu: float, h: float, fe_kind: int,
                      kind: int, M: int, tol: float = 1e-14, maxit: int = 50) -> np.ndarray:
    """Collocation solution by Newton's method on the full M*N-by-M*N system.

    Sec. 1: U_m = u_0 + dt sum_j q_{m,j} f(U_j) for all m at once, with
    f = nu L_h + f^E.  Dense linear algebra, so only for tiny grids.
    Returns u(T_{n+1}): U_M, or u_0 + dt sum_j b_j f(U_j) for Gauss-Legendre.
    """
    from .operators import f_explicit, laplacian, laplacian_matrix, f_explicit_derivative

    shape = u0.shape
    N = u0.size
    Q = qmatrix(kind, M)
    Lm = laplacian_matrix(shape[0], u0.ndim, h)
    U = np.tile(u0.reshape(1, N), (M, 1))
    for _ in range(maxit):
        F = np.stack([nu * laplacian(U[j].reshape(shape), h).reshape(N)
                      + f_explicit(U[j].reshape(shape), fe_kind).reshape(N) for j in range(M)])
        G = U - u0.reshape(1, N) - dt * (Q @ F)
        J = np.eye(M * N)
        for m in range(M):
            for j in range(M):
                if Q[m, j] != 0.0:
                    Jf = nu * Lm + np.diag(f_explicit_derivative(U[j], fe_kind))
                    J[m * N:(m + 1) * N, j * N:(j + 1) * N] -= dt * Q[m, j] * Jf
        delta = np.linalg.solve(J, G.reshape(M * N))
        U = U - delta.reshape(M, N)
        if np.max(np.abs(delta)) < tol:
            break
    if ends_on_node(kind):
        return U[-1].reshape(shape)
    F = np.stack([nu * laplacian(U[j].reshape(shape), h).reshape(N)
                  + f_explicit(U[j].reshape(shape), fe_kind).reshape(N) for j in range(M)])
    return (u0.reshape(N) + dt * (end_weights(kind, M) @ F)).reshape(shape)
