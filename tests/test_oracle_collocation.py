"""Pins for the oracle's nodes, quadrature matrices and collocation solutions.

Each expected value comes from a closed form or a textbook tableau, never from
the oracle itself.
"""

import math

import numpy as np
import pytest

import oracle as O
from oracle.collocation import NODES_LOBATTO as LOB, NODES_RADAU_RIGHT as RAD, NODES_LEGENDRE as LEG


# ---- nodes: closed forms of the Gauss-Lobatto / right Gauss-Radau points ----

def test_lobatto_nodes_closed_form():
    np.testing.assert_allclose(O.nodes(LOB, 2), [0.0, 1.0], atol=0, rtol=0)
    np.testing.assert_allclose(O.nodes(LOB, 3), [0.0, 0.5, 1.0], atol=1e-16)
    x = 1.0 / math.sqrt(5.0)
    np.testing.assert_allclose(O.nodes(LOB, 4), [0, (1 - x) / 2, (1 + x) / 2, 1], atol=1e-16)
    x = math.sqrt(3.0 / 7.0)
    np.testing.assert_allclose(O.nodes(LOB, 5), [0, (1 - x) / 2, 0.5, (1 + x) / 2, 1], atol=1e-16)
    # 7 points: interior roots of P_6' satisfy x^2 = (15 -+ 2 sqrt 15) / 33 and x = 0
    a = math.sqrt((15 - 2 * math.sqrt(15)) / 33)
    b = math.sqrt((15 + 2 * math.sqrt(15)) / 33)
    expect = [0, (1 - b) / 2, (1 - a) / 2, 0.5, (1 + a) / 2, (1 + b) / 2, 1]
    np.testing.assert_allclose(O.nodes(LOB, 7), expect, atol=2e-16)


def test_radau_right_nodes_closed_form():
    np.testing.assert_allclose(O.nodes(RAD, 1), [1.0], atol=0)
    np.testing.assert_allclose(O.nodes(RAD, 2), [1.0 / 3.0, 1.0], atol=1e-16)
    s6 = math.sqrt(6.0)
    np.testing.assert_allclose(O.nodes(RAD, 3), [(4 - s6) / 10, (4 + s6) / 10, 1.0], atol=1e-16)


@pytest.mark.parametrize("kind", [LOB, RAD])
@pytest.mark.parametrize("M", [2, 3, 4, 5, 6, 7, 8, 9])
def test_nodes_sorted_in_unit_interval(kind, M):
    if kind == LOB and M < 2:
        pytest.skip()
    t = O.nodes(kind, M)
    assert len(t) == M
    assert np.all(np.diff(t) > 0)
    assert t[-1] == 1.0
    assert t[0] >= 0.0
    if kind == LOB:
        assert t[0] == 0.0
    else:
        assert t[0] > 0.0


# ---- quadrature: polynomial exactness and textbook tableaux ----

@pytest.mark.parametrize("kind", [LOB, RAD])
@pytest.mark.parametrize("M", [2, 3, 4, 5, 6, 7, 8, 9])
def test_q_integrates_polynomials_exactly(kind, M):
    tau = O.nodes(kind, M)
    Q = O.qmatrix(kind, M)
    for p in range(M):  # degree <= M-1 is reproduced exactly by the interpolant
        lhs = Q @ tau ** p
        rhs = tau ** (p + 1) / (p + 1)
        np.testing.assert_allclose(lhs, rhs, atol=2e-15, rtol=0)


def test_q_lobatto3_is_lobatto_iiia():
    # Lobatto IIIA (3 stages), the standard Butcher tableau
    expect = np.array([[0, 0, 0], [5 / 24, 1 / 3, -1 / 24], [1 / 6, 2 / 3, 1 / 6]])
    np.testing.assert_allclose(O.qmatrix(LOB, 3), expect, atol=2e-16)


def test_q_radau3_is_radau_iia():
    s6 = math.sqrt(6.0)
    expect = np.array([
        [(88 - 7 * s6) / 360, (296 - 169 * s6) / 1800, (-2 + 3 * s6) / 225],
        [(296 + 169 * s6) / 1800, (88 + 7 * s6) / 360, (-2 - 3 * s6) / 225],
        [(16 - s6) / 36, (16 + s6) / 36, 1 / 9],
    ])
    np.testing.assert_allclose(O.qmatrix(RAD, 3), expect, atol=1e-15)


def test_lobatto5_weights():
    # last row of Q = quadrature weights on [0, 1]: half the classical 5-point
    # Gauss-Lobatto weights 1/10, 49/90, 32/45, 49/90, 1/10 on [-1, 1]
    expect = np.array([1 / 20, 49 / 180, 16 / 45, 49 / 180, 1 / 20])
    np.testing.assert_allclose(O.qmatrix(LOB, 5)[-1], expect, atol=2e-16)


@pytest.mark.parametrize("kind", [LOB, RAD])
@pytest.mark.parametrize("M", [2, 3, 5, 7, 9])
def test_s_rows_are_node_to_node_integrals(kind, M):
    tau = O.nodes(kind, M)
    S = O.smatrix(kind, M)
    Q = O.qmatrix(kind, M)
    tau_ext = np.concatenate([[0.0], tau])
    # S_m^{m+1} applied to f = 1 gives the substep length
    np.testing.assert_allclose(S.sum(axis=1), np.diff(tau_ext), atol=2e-16)
    # cumulative sums of S rows rebuild Q
    np.testing.assert_allclose(np.cumsum(S, axis=0), Q, atol=3e-16)
    # integral of s^p over [tau_m, tau_{m+1}] for p <= M-1
    for p in range(M):
        np.testing.assert_allclose(S @ tau ** p, np.diff(tau_ext ** (p + 1)) / (p + 1), atol=2e-15)
    if kind == LOB:
        assert np.all(S[0] == 0.0)


# ---- collocation stability functions: the Pade forms ----

def _pade_lobatto3(z):
    return (1 + z / 2 + z * z / 12) / (1 - z / 2 + z * z / 12)


def _pade_lobatto5(z):
    num = 1 + z / 2 + 3 * z ** 2 / 28 + z ** 3 / 84 + z ** 4 / 1680
    den = 1 - z / 2 + 3 * z ** 2 / 28 - z ** 3 / 84 + z ** 4 / 1680
    return num / den


def _pade_radau3(z):
    return (1 + 2 * z / 5 + z * z / 20) / (1 - 3 * z / 5 + 3 * z * z / 20 - z ** 3 / 60)


@pytest.mark.parametrize("kind,M,R", [(LOB, 3, _pade_lobatto3), (LOB, 5, _pade_lobatto5),
                                      (RAD, 3, _pade_radau3)])
def test_stability_function_is_pade(kind, M, R):
    z = np.array([0.0, -0.01, -0.5, -1.0, -3.0, -10.0, -100.0, -655.0, 0.3])
    np.testing.assert_allclose(O.stability_function(z, kind, M), R(z), rtol=2e-14, atol=1e-15)


def test_stability_function_order():
    # collocation order 2M-2 (Lobatto) / 2M-1 (Radau): R(z) - e^z = O(z^{p+1})
    for kind, M, p, z1 in [(LOB, 3, 4, -0.1), (LOB, 5, 8, -0.5), (RAD, 3, 5, -0.2)]:
        z2 = z1 / 2
        e1 = abs(O.stability_function(z1, kind, M) - math.exp(z1))
        e2 = abs(O.stability_function(z2, kind, M) - math.exp(z2))
        assert 2 ** (p + 1) * 0.6 < e1 / e2 < 2 ** (p + 1) * 1.3


# ---- direct collocation solves agree with each other and with closed forms ----

def _sine_u0(n, d, modes):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    u = np.zeros((n,) * d)
    for amp, a in modes:
        term = amp * np.ones((n,) * d)
        for ax in range(d):
            shape = [1] * d
            shape[ax] = n
            term = term * np.sin(a[ax] * np.pi * x).reshape(shape)
        u = u + term
    return u, h


def test_modal_collocation_closed_form_1d():
    # u0 = sin(pi x) + 0.5 sin(3 pi x), n = 127, dt = 0.01, nu = 1, Lobatto M = 3:
    # each mode is multiplied by R(dt * lambda_a) with
    # lambda_a = -(4/h^2) sin^2(a pi h / 2)
    n = 127
    u0, h = _sine_u0(n, 1, [(1.0, (1,)), (0.5, (3,))])
    x = (np.arange(n) + 1) * h
    lam1 = -(4 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    lam3 = -(4 / h ** 2) * math.sin(3 * math.pi * h / 2) ** 2
    assert abs(lam1 - (-9.869108962780)) < 1e-11
    assert abs(lam3 - (-88.78631555268)) < 1e-10
    expect = (_pade_lobatto3(0.01 * lam1) * np.sin(np.pi * x)
              + 0.5 * _pade_lobatto3(0.01 * lam3) * np.sin(3 * np.pi * x))
    got = O.collocation_heat_modal(u0, 0.01, 1.0, h, LOB, 3)
    np.testing.assert_allclose(got, expect, atol=2e-15)


@pytest.mark.parametrize("d,n,kind,M", [(1, 15, LOB, 3), (2, 7, LOB, 5), (2, 7, RAD, 3), (3, 3, LOB, 3)])
def test_dense_collocation_equals_modal_for_heat(d, n, kind, M):
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((n,) * d)
    h = 1.0 / (n + 1)
    dense = O.collocation_dense(u0, 0.02, 0.7, h, O.FE_ZERO, kind, M)
    modal = O.collocation_heat_modal(u0, 0.02, 0.7, h, kind, M)
    np.testing.assert_allclose(dense, modal, atol=1e-13)


def test_pointwise_ode_closed_form():
    # nu = 0 with f^E = u - u^3: each point solves u' = u - u^3, whose exact
    # solution is u0 e^t / sqrt(1 - u0^2 + u0^2 e^{2t}); Lobatto M = 5 has order 8
    u0 = np.array([[0.3, -0.7, 0.05], [0.9, -0.2, 0.5], [0.0, 1.0, -1.0]])
    dt = 0.1
    got = O.collocation_dense(u0, dt, 0.0, 0.25, O.FE_CUBIC, LOB, 5)
    expect = u0 * math.exp(dt) / np.sqrt(1 - u0 ** 2 + u0 ** 2 * math.exp(2 * dt))
    np.testing.assert_allclose(got, expect, atol=1e-11)


# ---- Gauss-Legendre nodes: interior points, end value by the quadrature ----

def test_legendre_nodes_and_weights_closed_form():
    r3, r15 = math.sqrt(3.0), math.sqrt(15.0)
    np.testing.assert_allclose(O.nodes(LEG, 1), [0.5], atol=1e-16)
    np.testing.assert_allclose(O.nodes(LEG, 2), [0.5 - r3 / 6, 0.5 + r3 / 6], atol=1e-16)
    np.testing.assert_allclose(O.nodes(LEG, 3), [0.5 - r15 / 10, 0.5, 0.5 + r15 / 10], atol=1e-16)
    np.testing.assert_allclose(O.end_weights(LEG, 1), [1.0], atol=1e-16)
    np.testing.assert_allclose(O.end_weights(LEG, 2), [0.5, 0.5], atol=1e-16)
    np.testing.assert_allclose(O.end_weights(LEG, 3), [5 / 18, 4 / 9, 5 / 18], atol=1e-16)


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 7, 9])
def test_legendre_quadrature_exact_to_degree_2m_minus_1(M):
    # Gauss quadrature: the end weights integrate s^p over [0, 1] exactly for
    # p <= 2M - 1, which only the roots of P_M achieve; Q still integrates
    # degree <= M - 1 up to every node
    tau, b, Q = O.nodes(LEG, M), O.end_weights(LEG, M), O.qmatrix(LEG, M)
    assert np.all(tau > 0) and np.all(tau < 1) and np.all(np.diff(tau) > 0)
    for p in range(2 * M):
        assert abs(b @ tau ** p - 1.0 / (p + 1)) < 4e-15
    for p in range(M):
        np.testing.assert_allclose(Q @ tau ** p, tau ** (p + 1) / (p + 1), atol=2e-15)
    S = O.smatrix(LEG, M)
    np.testing.assert_allclose(np.cumsum(S, axis=0), Q, atol=3e-16)
    assert np.all(np.abs(S[0]) > 0)  # tau_1 > 0: no degenerate first substep


def test_end_weights_are_last_q_row_where_tau_m_is_one():
    for kind, M in [(LOB, 3), (LOB, 6), (RAD, 2), (RAD, 5)]:
        np.testing.assert_allclose(O.end_weights(kind, M), O.qmatrix(kind, M)[-1], atol=2e-16)


def test_q_legendre_is_gauss_tableau():
    r3, r15 = math.sqrt(3.0), math.sqrt(15.0)
    np.testing.assert_allclose(O.qmatrix(LEG, 2), [[0.25, 0.25 - r3 / 6], [0.25 + r3 / 6, 0.25]], atol=2e-16)
    ref = [[5 / 36, 2 / 9 - r15 / 15, 5 / 36 - r15 / 30],
           [5 / 36 + r15 / 24, 2 / 9, 5 / 36 - r15 / 24],
           [5 / 36 + r15 / 30, 2 / 9 + r15 / 15, 5 / 36]]
    np.testing.assert_allclose(O.qmatrix(LEG, 3), ref, atol=3e-16)


def _pade_gauss(M):
    # diagonal (M, M) Pade approximant of e^z
    def coef(k):
        return math.factorial(2 * M - k) * math.factorial(M) / (math.factorial(2 * M) * math.factorial(k)
                                                               * math.factorial(M - k))

    def R(z):
        num = sum(coef(k) * z ** k for k in range(M + 1))
        den = sum(coef(k) * (-z) ** k for k in range(M + 1))
        return num / den
    return R


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_legendre_stability_function_is_diagonal_pade(M):
    z = np.array([0.0, -0.01, -0.5, -1.0, -3.0, -10.0, -100.0, 0.3])
    np.testing.assert_allclose(O.stability_function(z, LEG, M), _pade_gauss(M)(z), rtol=2e-14, atol=1e-15)
    if M == 3:  # written out: (1 + z/2 + z^2/10 + z^3/120) / (1 - z/2 + z^2/10 - z^3/120)
        zz = -2.5
        ref = (1 + zz / 2 + zz ** 2 / 10 + zz ** 3 / 120) / (1 - zz / 2 + zz ** 2 / 10 - zz ** 3 / 120)
        assert abs(O.stability_function(zz, LEG, 3) - ref) < 1e-15


def test_legendre_order_2m():
    for M, z1 in [(2, -0.2), (3, -0.6)]:
        e1 = abs(O.stability_function(z1, LEG, M) - math.exp(z1))
        e2 = abs(O.stability_function(z1 / 2, LEG, M) - math.exp(z1 / 2))
        assert 2 ** (2 * M + 1) * 0.6 < e1 / e2 < 2 ** (2 * M + 1) * 1.3


@pytest.mark.parametrize("d,n,M", [(1, 15, 3), (2, 7, 2)])
def test_legendre_dense_collocation_equals_modal_for_heat(d, n, M):
    rng = np.random.default_rng(12)
    u0 = rng.standard_normal((n,) * d)
    h = 1.0 / (n + 1)
    dense = O.collocation_dense(u0, 0.02, 0.7, h, O.FE_ZERO, LEG, M)
    modal = O.collocation_heat_modal(u0, 0.02, 0.7, h, LEG, M)
    np.testing.assert_allclose(dense, modal, atol=1e-13)


def test_legendre_pointwise_ode_order():
    # nu = 0, u' = u - u^3 pointwise: Gauss M = 3 has order 6 at the end point
    u0 = np.array([[0.3, -0.7], [0.9, 0.05]])
    errs = []
    for dt in (0.4, 0.2):
        got = O.collocation_dense(u0, dt, 0.0, 0.25, O.FE_CUBIC, LEG, 3)
        expect = u0 * math.exp(dt) / np.sqrt(1 - u0 ** 2 + u0 ** 2 * math.exp(2 * dt))
        errs.append(np.max(np.abs(got - expect)))
    assert errs[1] < 1e-7 and 2 ** 7 * 0.5 < errs[0] / errs[1] < 2 ** 7 * 1.5


def _pade_exp(k, j):
    """(k, j) Pade approximant of exp from its textbook coefficients."""
    f = math.factorial
    num = [f(k + j - i) * f(k) / (f(k + j) * f(i) * f(k - i)) for i in range(k + 1)]
    den = [(-1) ** i * f(k + j - i) * f(j) / (f(k + j) * f(i) * f(j - i)) for i in range(j + 1)]
    return lambda z: np.polyval(num[::-1], z) / np.polyval(den[::-1], z)


@pytest.mark.parametrize("kind,Ms", [(LOB, range(2, 10)), (RAD, range(1, 10)), (LEG, range(1, 10))])
def test_stability_function_is_pade_for_every_m(kind, Ms):
    # Lobatto IIIA: (M-1, M-1) Pade; Radau IIA: (M-1, M); Gauss: (M, M)
    z = np.array([0.0, -0.01, -0.5, -1.0, -3.0, -10.0, -100.0, -655.0, 0.3])
    for M in Ms:
        k, j = {LOB: (M - 1, M - 1), RAD: (M - 1, M), LEG: (M, M)}[kind]
        np.testing.assert_allclose(O.stability_function(z, kind, M), _pade_exp(k, j)(z), rtol=1e-13, atol=1e-15)
