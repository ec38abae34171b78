"""Pins for the oracle's operators and multigrid V-cycle.

Expected values come from trigonometric identities, brute-force loops written
independently here, adjointness and Galerkin identities, and direct solves.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.multigrid import residual_inf


def _grid(n):
    h = 1.0 / (n + 1)
    return (np.arange(n) + 1) * h, h


def _sine(n, d, a):
    x, h = _grid(n)
    u = np.ones((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        u = u * np.sin(a[ax] * np.pi * x).reshape(shape)
    return u, h


# ---- Laplacian ----

@pytest.mark.parametrize("d,n,a", [(1, 15, (3,)), (2, 15, (1, 4)), (3, 7, (2, 1, 5)), (2, 31, (31, 1))])
def test_laplacian_sine_mode_eigenvalue(d, n, a):
    # trig identity: sin(k(x-h)) - 2 sin(kx) + sin(k(x+h)) = -4 sin^2(kh/2) sin(kx);
    # the zero ghosts coincide with sin(k*0) = sin(k*1) = 0 for integer a
    u, h = _sine(n, d, a)
    lam = sum(-4.0 / h ** 2 * math.sin(ai * math.pi * h / 2) ** 2 for ai in a)
    np.testing.assert_allclose(O.laplacian(u, h), lam * u, atol=1e-10 * abs(lam))
    eig = O.laplacian_eigenvalues(n, d, h)
    assert abs(eig[tuple(ai - 1 for ai in a)] - lam) < 1e-12 * abs(lam)


def test_laplacian_second_order_consistency():
    # L_h sin(pi x) sin(pi y) -> -2 pi^2 sin(pi x) sin(pi y) with O(h^2) error
    errs = []
    for n in (15, 31, 63):
        u, h = _sine(n, 2, (1, 1))
        errs.append(np.max(np.abs(O.laplacian(u, h) + 2 * math.pi ** 2 * u)))
    assert 3.7 < errs[0] / errs[1] < 4.3 and 3.7 < errs[1] / errs[2] < 4.3


def test_laplacian_brute_force_loops():
    rng = np.random.default_rng(3)
    n, h = 5, 0.25
    u = rng.standard_normal((n, n, n))

    def at(i, j, k):
        if min(i, j, k) < 0 or max(i, j, k) >= n:
            return 0.0
        return u[i, j, k]

    ref = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                s = (at(i - 1, j, k) + at(i + 1, j, k) + at(i, j - 1, k) + at(i, j + 1, k)
                     + at(i, j, k - 1) + at(i, j, k + 1) - 6 * u[i, j, k])
                ref[i, j, k] = s / h ** 2
    np.testing.assert_allclose(O.laplacian(u, h), ref, atol=1e-12)
    from oracle.operators import laplacian_matrix
    np.testing.assert_allclose(laplacian_matrix(n, 3, h) @ u.reshape(-1), ref.reshape(-1), atol=1e-11)


def test_exact_shifted_solve():
    rng = np.random.default_rng(4)
    for d, n in [(1, 31), (2, 15), (3, 7)]:
        x, h = _grid(n)
        rhs = rng.standard_normal((n,) * d)
        c = 0.37
        u = O.solve_shifted_exact(rhs, c, h)
        np.testing.assert_allclose(O.apply_shifted(u, c, h), rhs, atol=1e-12)
        from oracle.operators import laplacian_matrix
        dense = np.linalg.solve(np.eye(n ** d) - c * laplacian_matrix(n, d, h), rhs.reshape(-1))
        np.testing.assert_allclose(u.reshape(-1), dense, atol=1e-12)


def test_f_explicit():
    u = np.array([-2.0, -1.0, 0.0, 0.5, 1.0, 3.0])
    np.testing.assert_array_equal(O.f_explicit(u, O.FE_ZERO), np.zeros(6))
    np.testing.assert_allclose(O.f_explicit(u, O.FE_CUBIC), [6.0, 0.0, 0.0, 0.375, 0.0, -24.0])


# ---- transfer operators ----

def test_level_sizes():
    assert O.level_sizes(1) == [1]
    assert O.level_sizes(7) == [7, 3, 1]
    assert O.level_sizes(1023) == [1023, 511, 255, 127, 63, 31, 15, 7, 3, 1]
    with pytest.raises(ValueError):
        O.level_sizes(10)


@pytest.mark.parametrize("d,n", [(1, 15), (2, 7), (3, 7)])
def test_restriction_is_scaled_adjoint_of_prolongation(d, n):
    # full weighting and linear interpolation satisfy P = 2^d R^T
    rng = np.random.default_rng(5)
    nc = (n - 1) // 2
    r = rng.standard_normal((n,) * d)
    ec = rng.standard_normal((nc,) * d)
    lhs = (2 ** d) * np.sum(O.restrict_fw(r) * ec)
    rhs = np.sum(r * O.prolong_linear(ec))
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_transfer_brute_force_1d():
    rng = np.random.default_rng(6)
    n = 15
    nc = 7
    r = rng.standard_normal(n)
    ec = rng.standard_normal(nc)
    rc = np.array([0.25 * r[2 * i] + 0.5 * r[2 * i + 1] + 0.25 * r[2 * i + 2] for i in range(nc)])
    np.testing.assert_allclose(O.restrict_fw(r), rc, atol=1e-15)
    ecp = np.concatenate([[0.0], ec, [0.0]])
    e = np.zeros(n)
    for i in range(n):
        if i % 2 == 1:
            e[i] = ec[(i - 1) // 2]
        else:
            e[i] = 0.5 * (ecp[i // 2] + ecp[i // 2 + 1])
    np.testing.assert_allclose(O.prolong_linear(ec), e, atol=1e-15)


def test_galerkin_identity_1d():
    # in 1D, R L_h P equals the rediscretised L_{2h} for these transfers
    n = 15
    h = 1.0 / (n + 1)
    nc = 7
    cols = []
    for i in range(nc):
        ec = np.zeros(nc)
        ec[i] = 1.0
        cols.append(O.restrict_fw(O.laplacian(O.prolong_linear(ec), h)))
    RLP = np.stack(cols, axis=1)
    from oracle.operators import laplacian_matrix
    np.testing.assert_allclose(RLP, laplacian_matrix(nc, 1, 2 * h), atol=1e-10)


def test_full_weighting_second_order():
    # FW of a smooth function matches it at the coarse points up to O(h^2)
    errs = []
    for n in (31, 63, 127):
        x, h = _grid(n)
        f = np.exp(x) * np.sin(np.pi * x)
        xc = x[1::2]
        errs.append(np.max(np.abs(O.restrict_fw(f) - np.exp(xc) * np.sin(np.pi * xc))))
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


# ---- smoothers against brute-force loops ----

def test_rbgs_matches_sequential_loop_2d():
    rng = np.random.default_rng(7)
    n = 7
    x, h = _grid(n)
    c = 0.013
    u = rng.standard_normal((n, n))
    rhs = rng.standard_normal((n, n))
    a = c / h ** 2
    v = u.copy()
    for colour in (0, 1):  # red (even i+j) first, one point at a time
        for i in range(n):
            for j in range(n):
                if (i + j) % 2 != colour:
                    continue
                s = 0.0
                for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                    ii, jj = i + di, j + dj
                    if 0 <= ii < n and 0 <= jj < n:
                        s += v[ii, jj]
                v[i, j] = (rhs[i, j] + a * s) / (1 + 4 * a)
    np.testing.assert_allclose(O.smooth(u, rhs, c, h, O.SMOOTH_RBGS), v, atol=1e-13)


def test_jacobi_matches_loop_3d():
    rng = np.random.default_rng(8)
    n = 3
    x, h = _grid(n)
    c = 0.05
    u = rng.standard_normal((n, n, n))
    rhs = rng.standard_normal((n, n, n))
    a = c / h ** 2
    D = 1 + 6 * a
    out = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                s = 0.0
                for dv in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    p = (i + dv[0], j + dv[1], k + dv[2])
                    if all(0 <= q < n for q in p):
                        s += u[p]
                Au = D * u[i, j, k] - a * s
                out[i, j, k] = u[i, j, k] + (6 / 7) * (rhs[i, j, k] - Au) / D
    np.testing.assert_allclose(O.smooth(u, rhs, c, h, O.SMOOTH_JACOBI), out, atol=1e-12)


# ---- V-cycle ----

@pytest.mark.parametrize("smoother,nu1,nu2", [(O.SMOOTH_RBGS, 1, 1), (O.SMOOTH_JACOBI, 2, 2)])
@pytest.mark.parametrize("d,n", [(1, 63), (2, 31), (3, 15)])
def test_vcycle_fixed_point_and_convergence(smoother, nu1, nu2, d, n):
    rng = np.random.default_rng(9)
    x, h = _grid(n)
    c = 40 * h * h
    rhs = rng.standard_normal((n,) * d)
    exact = O.solve_shifted_exact(rhs, c, h)
    # the exact solution is a fixed point of the cycle
    np.testing.assert_allclose(O.vcycle(exact, rhs, c, h, smoother, nu1, nu2), exact, atol=1e-12)
    # cycles converge to the exact solution
    u = np.zeros_like(rhs)
    for _ in range(25):
        u = O.vcycle(u, rhs, c, h, smoother, nu1, nu2)
    np.testing.assert_allclose(u, exact, atol=1e-11 * np.max(np.abs(exact)))


def test_vcycle_affine_u_form_equals_e_form():
    rng = np.random.default_rng(10)
    n = 31
    x, h = _grid(n)
    c = 80 * h * h
    rhs = rng.standard_normal((n, n))
    g = rng.standard_normal((n, n))
    u_form = O.vcycle(g, rhs, c, h)
    e_form = g + O.vcycle(np.zeros_like(g), rhs - O.apply_shifted(g, c, h), c, h)
    np.testing.assert_allclose(u_form, e_form, atol=1e-12)


def _iteration_matrix(n, d, c, smoother, nu1, nu2):
    h = 1.0 / (n + 1)
    N = n ** d
    cols = []
    z = np.zeros((n,) * d)
    for i in range(N):
        e = np.zeros(N)
        e[i] = 1.0
        cols.append(O.vcycle(e.reshape((n,) * d), z, c, h, smoother, nu1, nu2).reshape(-1))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("d,n,stiff", [(1, 31, 50.0), (2, 15, 50.0), (2, 15, 1.0), (3, 7, 20.0)])
def test_vcycle_contraction_matches_iteration_matrix(d, n, stiff):
    h = 1.0 / (n + 1)
    c = stiff * h * h
    E = _iteration_matrix(n, d, c, O.SMOOTH_RBGS, 1, 1)
    rho = max(abs(np.linalg.eigvals(E)))
    # power iteration with the oracle's cycle on the homogeneous problem
    rng = np.random.default_rng(12)
    e = rng.standard_normal((n,) * d)
    z = np.zeros_like(e)
    est = 0.0
    for _ in range(200):
        e2 = O.vcycle(e, z, c, h)
        est = np.linalg.norm(e2) / np.linalg.norm(e)
        e = e2 / np.linalg.norm(e2)
    assert abs(est - rho) < 1e-6 * rho + 1e-12
    # sanity band only (textbook RB-GS V(1,1) factors are ~0.05-0.25), not a pin
    assert 0.0 < rho < 0.35


def test_vcycle_float32_stays_float32():
    rng = np.random.default_rng(13)
    n = 63
    x, h = _grid(n)
    c = 50 * h * h
    rhs = rng.standard_normal((n, n))
    u64 = O.vcycle(np.zeros((n, n)), rhs, c, h)
    u32 = O.vcycle(np.zeros((n, n), np.float32), rhs.astype(np.float32), c, h)
    assert u32.dtype == np.float32
    np.testing.assert_allclose(u32, u64, atol=2e-6 * np.max(np.abs(u64)))


def test_residual_inf():
    n = 15
    x, h = _grid(n)
    u = np.zeros((n, n))
    rhs = np.zeros((n, n))
    rhs[3, 4] = -2.5
    assert residual_inf(u, rhs, 0.1, h) == 2.5
