"""Pins for the oracle's periodic compact stencil, periodic multigrid, WENO5
Burgers advection and the periodic Burgers sweep (Sec. 4.1, eq. (5)).

Targets that do not reuse the oracle's own formulas: stencils as loops with
modular indices, Fourier-mode eigenvalues in closed form, O(h^4) consistency,
dense solves, the linear fifth-order upwind flux that WENO5 reduces to when
its smoothness weights are switched off, the smoothness indicators and
candidate values recomputed from their integral and cell-average
definitions, the ENO property at a jump, discrete conservation, a
high-accuracy ODE integration (scipy DOP853) of the same semi-discrete
system, and the modal collocation solution of the periodic heat problem.
"""

import numpy as np
import pytest

import oracle as O
from oracle import periodic as P
from oracle.sdc import SDCConfig, sdc_step, sdc_begin, sdc_sweep, STENCIL_COMPACT4, BC_PERIODIC, FE_BURGERS

LOB = O.NODES_LOBATTO


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def _dense(op, n, d):
    N = n ** d
    cols = []
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        cols.append(op(e.reshape((n,) * d)).reshape(-1))
    return np.stack(cols, axis=1)


def test_periodic_stencils_are_wrapped_loops():
    n, h = 6, 0.3
    u = _rand((n, n), 1)
    lap = np.zeros_like(u)
    lapc = np.zeros_like(u)
    w = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            e = u[(i - 1) % n, j] + u[(i + 1) % n, j] + u[i, (j - 1) % n] + u[i, (j + 1) % n]
            c = (u[(i - 1) % n, (j - 1) % n] + u[(i - 1) % n, (j + 1) % n] + u[(i + 1) % n, (j - 1) % n]
                 + u[(i + 1) % n, (j + 1) % n])
            lap[i, j] = (e - 4 * u[i, j]) / h ** 2
            lapc[i, j] = (4 * e + c - 20 * u[i, j]) / (6 * h * h)
            w[i, j] = (8 * u[i, j] + e) / 12.0
    assert np.max(np.abs(P.laplacian_p(u, h) - lap)) < 1e-11
    assert np.max(np.abs(P.laplacian_compact_p(u, h) - lapc)) < 1e-11
    assert np.max(np.abs(P.weight_p(u, h) - w)) < 1e-14


def test_periodic_eigenvalues_closed_form():
    n = 16
    x, h = P.grid_p(n)
    lam_l, lam_a, lam_w = P.eigenvalues_p(n, 2, h)
    for a, b in [(0, 0), (1, 3), (8, 8), (5, 11)]:
        mode = np.outer(np.cos(np.pi * a * (x + 1)), np.cos(np.pi * b * (x + 1)))
        th, ph = 2 * np.pi * a / n, 2 * np.pi * b / n
        la = (8 * np.cos(th) + 8 * np.cos(ph) + 4 * np.cos(th) * np.cos(ph) - 20) / (6 * h * h)
        lw = (8 + 2 * np.cos(th) + 2 * np.cos(ph)) / 12.0
        assert abs(lam_a[a, b] - la) < 1e-9 * max(1.0, abs(la))
        assert abs(lam_w[a, b] - lw) < 1e-14
        assert np.max(np.abs(P.laplacian_compact_p(mode, h) - la * mode)) < 1e-9 * max(1.0, abs(la))


def test_periodic_fourth_order():
    errs = []
    for n in (16, 32, 64):
        x, h = P.grid_p(n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        u = np.sin(np.pi * X) * np.cos(2 * np.pi * Y)
        exact = -5 * np.pi ** 2 * u
        errs.append(np.max(np.abs(P.solve_weight_exact_p(P.laplacian_compact_p(u, h), h) - exact)))
    assert 14 < errs[0] / errs[1] < 18 and 14 < errs[1] / errs[2] < 18


def test_periodic_exact_solves_against_dense():
    n, h, c = 6, 0.25, 0.02
    rhs = _rand((n, n), 2)
    B = _dense(lambda v: P.weight_p(v, h) - c * P.laplacian_compact_p(v, h), n, 2)
    W = _dense(lambda v: P.weight_p(v, h), n, 2)
    assert np.max(np.abs(P.solve_compact_shifted_exact_p(rhs, c, h) - np.linalg.solve(B, rhs.reshape(-1)).reshape(n, n))) < 1e-12
    assert np.max(np.abs(P.solve_weight_exact_p(rhs, h) - np.linalg.solve(W, rhs.reshape(-1)).reshape(n, n))) < 1e-12
    assert abs(P.compact_diagonal_p(2, c, h * h / 12, h) - B[0, 0]) < 1e-12


def test_periodic_transfers_are_loops_and_adjoint():
    n = 8
    r = _rand((n, n), 3)
    rc = np.zeros((n // 2, n // 2))
    wts = {-1: 0.25, 0: 0.5, 1: 0.25}
    for I in range(n // 2):
        for J in range(n // 2):
            rc[I, J] = sum(wts[a] * wts[b] * r[(2 * I + a) % n, (2 * J + b) % n] for a in (-1, 0, 1) for b in (-1, 0, 1))
    assert np.max(np.abs(P.restrict_fw_p(r) - rc)) < 1e-14
    ec = _rand((n // 2, n // 2), 4)
    e = P.prolong_linear_p(ec)
    assert abs(e[2, 4] - ec[1, 2]) < 1e-15
    assert abs(e[3, 4] - 0.5 * (ec[1, 2] + ec[2, 2])) < 1e-15
    assert abs(e[7, 7] - 0.25 * (ec[3, 3] + ec[0, 3] + ec[3, 0] + ec[0, 0])) < 1e-15
    R = _dense(P.restrict_fw_p, n, 2)
    Pm = _dense(P.prolong_linear_p, n // 2, 2)
    assert np.allclose(Pm, 4 * R.T)


@pytest.mark.parametrize("c_h2", [0.4, 40.0])
def test_periodic_vcycle_converges(c_h2):
    n = 64
    x, h = P.grid_p(n)
    c = c_h2 * h * h
    rhs = _rand((n, n), 5)
    exact = P.solve_compact_shifted_exact_p(rhs, c, h)
    u = np.zeros_like(rhs)
    errs = []
    for _ in range(6):
        u = P.vcycle_compact_p(u, rhs, c, h, 3, 3)
        errs.append(np.max(np.abs(u - exact)))
    assert errs[3] / errs[2] < 0.15 and errs[-1] < 1e-6 * np.max(np.abs(exact))
    n2, h2 = 8, 0.25
    G = _dense(lambda e0: P.vcycle_compact_p(e0, np.zeros((n2, n2)), c_h2 * h2 * h2, h2, 3, 3), n2, 2)
    assert max(abs(np.linalg.eigvals(G))) < 0.2


def test_weno5_reduces_to_linear_upwind_flux():
    # with the smoothness indicators switched off (huge epsilon) the weights are
    # the linear ones and WENO5 is the fifth-order upwind flux
    # (2 f_{i-2} - 13 f_{i-1} + 47 f_i + 27 f_{i+1} - 3 f_{i+2}) / 60 for f^+ and its mirror for f^-
    n = 12
    u = 0.3 + _rand((n, n), 6) ** 2
    F = P.weno5_flux(u, 0, eps=1e40)
    ref = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            a = max(abs(u[i, j]), abs(u[(i + 1) % n, j]))
            fp = lambda k: 0.5 * (0.5 * u[(i + k) % n, j] ** 2 + a * u[(i + k) % n, j])  # noqa: E731
            fm = lambda k: 0.5 * (0.5 * u[(i + k) % n, j] ** 2 - a * u[(i + k) % n, j])  # noqa: E731
            ref[i, j] = ((2 * fp(-2) - 13 * fp(-1) + 47 * fp(0) + 27 * fp(1) - 3 * fp(2)) / 60.0
                         + (-3 * fm(-1) + 27 * fm(0) + 47 * fm(1) - 13 * fm(2) + 2 * fm(3)) / 60.0)
    assert np.max(np.abs(F - ref)) < 1e-12


def _jiang_shu_candidates(vals):
    """Independent evaluation of the Jiang-Shu WENO5 ingredients on one face,
    from their definitions rather than from the closed-form coefficients:
    for each candidate stencil k (cells i-2+k .. i+k, unit cells, cell i =
    [-1/2, 1/2]) the quadratic p_k whose cell averages equal the given values,
    its value at the face x = 1/2, and the smoothness indicator
    beta_k = sum_{l=1,2} integral over cell i of (d^l p_k / dx^l)^2
    (the h^(2l-1) factors are 1 on unit cells)."""
    from numpy.polynomial import polynomial as Pn
    q, beta = [], []
    for k in range(3):
        cells = [j - 2 + k for j in range(3)]
        # cell average of x^p over [j - 1/2, j + 1/2] is ((j+1/2)^(p+1) - (j-1/2)^(p+1)) / (p+1)
        A = np.array([[((j + 0.5) ** (p + 1) - (j - 0.5) ** (p + 1)) / (p + 1) for p in range(3)] for j in cells])
        coef = np.linalg.solve(A, np.asarray(vals[k:k + 3], dtype=np.float64))
        q.append(Pn.polyval(0.5, coef))
        b = 0.0
        for l in (1, 2):
            d = Pn.polyder(coef, l)
            sq = Pn.polyint(Pn.polymul(d, d))
            b += Pn.polyval(0.5, sq) - Pn.polyval(-0.5, sq)
        beta.append(b)
    return np.array(q), np.array(beta)


@pytest.mark.parametrize("seed", range(6))
def test_weno5_indicators_and_weights_follow_jiang_shu(seed):
    # smoothness indicators and candidate values from their integral and
    # cell-average definitions; the nonlinear weights d_k / (eps + beta_k)^2
    # with eps = 1e-6 (Jiang and Shu).  Values scaled so that beta ~ eps,
    # where the result depends on eps and on every indicator term.
    rng = np.random.default_rng(100 + seed)
    scale = 10.0 ** rng.uniform(-4, 0)
    vals = scale * rng.standard_normal(5)
    q, beta = _jiang_shu_candidates(vals)
    dlin = np.array([0.1, 0.6, 0.3])
    alpha = dlin / (1e-6 + beta) ** 2
    ref = float(np.dot(alpha, q) / alpha.sum())
    got = P._weno5_left(*vals)
    assert abs(got - ref) <= 1e-12 * max(1.0, np.max(np.abs(vals)))


def test_weno5_eno_property_at_a_jump():
    # data with a jump between the face's two cells: the stencils that cross
    # it carry weights of order eps^2 / beta^2, so the reconstruction equals
    # the smooth stencil's value to about 1e-11 (a larger eps would leak
    # O(1e-4) of the crossing stencils into it)
    for left, right in ((0.0, 1.0), (2.0, -1.0), (0.5, 0.5 + 3.0)):
        vals = [left, left, left, right, right]
        got = P._weno5_left(*vals)
        assert abs(got - left) < 1e-10 * max(1.0, abs(right - left))
    # a jump one cell further right: only the rightmost stencil crosses it
    vals = [0.0, 0.0, 0.0, 0.0, 1.0]
    q, beta = _jiang_shu_candidates(vals)
    assert beta[0] == 0.0 and beta[1] == 0.0 and beta[2] > 1.0
    assert abs(P._weno5_left(*vals)) < 1e-10


def test_weno5_eps_enters_where_indicators_vanish():
    # beta_1 = 0 (b = c = d) while beta_0 and beta_2 are of order eps: the
    # result moves with eps at O(1) of the candidate spread
    vals = np.array([1.0e-3, 0.0, 0.0, 0.0, -2.0e-3])
    q, beta = _jiang_shu_candidates(vals)
    assert beta[1] == 0.0 and 1e-7 < beta[0] < 1e-5 and 1e-7 < beta[2] < 1e-5
    dlin = np.array([0.1, 0.6, 0.3])
    for eps in (1e-6, 1e-5):
        alpha = dlin / (eps + beta) ** 2
        ref = float(np.dot(alpha, q) / alpha.sum())
        assert abs(P._weno5_left(*vals, eps=eps) - ref) < 1e-15
    assert abs(P._weno5_left(*vals) - P._weno5_left(*vals, eps=1e-5)) > 1e-6 * np.ptp(q)
    assert P.WENO_EPS == 1e-6


def test_weno5_conservative_and_consistent():
    n = 64
    x, h = P.grid_p(n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    u = np.exp(-(X ** 2 + Y ** 2) / 0.1 ** 2)
    adv = P.burgers_advection(u, h)
    assert abs(np.sum(adv)) < 1e-10 * np.sum(np.abs(adv))  # periodic flux differences telescope
    assert np.max(np.abs(P.burgers_advection(np.full((8, 8), 0.7), 0.25))) < 1e-14
    errs = []
    for n in (32, 64, 128):
        x, h = P.grid_p(n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        u = 1.0 + 0.25 * np.sin(np.pi * X) * np.sin(np.pi * Y)
        exact = -u * (0.25 * np.pi * np.cos(np.pi * X) * np.sin(np.pi * Y)
                      + 0.25 * np.pi * np.sin(np.pi * X) * np.cos(np.pi * Y))
        errs.append(np.max(np.abs(P.burgers_advection(u, h) - exact)))
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8  # at least third order near extrema


def test_burgers_sdc_matches_ode_integration():
    # the step reaches the exact solution of the semi-discrete system
    # u' = nu W^{-1} A_h u + f^E(u) within the collocation error of M = 5 (order 8)
    from scipy.integrate import solve_ivp
    n, nu, dt = 16, 0.5, 2e-3
    x, h = P.grid_p(n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    u0 = 0.5 + np.exp(-(X ** 2 + Y ** 2) / 0.3 ** 2)
    cfg = SDCConfig(nu=nu, fe_kind=FE_BURGERS, node_kind=LOB, M=5, inner="exact", tol=1e-14, max_sweeps=80,
                    stencil=STENCIL_COMPACT4, bc=BC_PERIODIC)
    u, st = sdc_step(u0, dt, h, cfg)
    assert st.status == "ok"

    def rhs(t, y):
        v = y.reshape(n, n)
        return (nu * P.solve_weight_exact_p(P.laplacian_compact_p(v, h), h) + P.burgers_advection(v, h)).reshape(-1)

    ref = solve_ivp(rhs, (0.0, dt), u0.reshape(-1), method="DOP853", rtol=1e-13, atol=1e-15).y[:, -1].reshape(n, n)
    assert np.max(np.abs(u - ref)) < 1e-11


def test_periodic_heat_reaches_modal_collocation():
    n, nu, dt, M = 32, 2.0, 2e-3, 5
    x, h = P.grid_p(n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    u0 = np.cos(np.pi * X) * np.sin(2 * np.pi * Y) + 0.2
    _, lam_a, lam_w = P.eigenvalues_p(n, 2, h)
    R = O.stability_function(dt * nu * lam_a / lam_w, LOB, M)
    coll = np.real(np.fft.ifftn(np.fft.fftn(u0) * R))
    for inner in ("exact", "mg"):
        cfg = SDCConfig(nu=nu, node_kind=LOB, M=M, inner=inner, tol=1e-13, smoother=1, nu1=3, nu2=3,
                        stencil=STENCIL_COMPACT4, bc=BC_PERIODIC, max_sweeps=100)
        u, st = sdc_step(u0, dt, h, cfg)
        assert st.status == "ok"
        assert np.linalg.norm(u - coll) / np.linalg.norm(coll) < 1e-11


def test_periodic_configuration_checks():
    u0 = np.zeros((8, 8))
    with pytest.raises(ValueError):
        sdc_begin(u0, 1e-3, 0.25, SDCConfig(bc=BC_PERIODIC))  # second-order periodic not provided
    with pytest.raises(ValueError):
        sdc_begin(u0, 1e-3, 0.25, SDCConfig(fe_kind=FE_BURGERS, stencil=STENCIL_COMPACT4))


def test_burgers_first_sweep_is_imex_euler():
    # right Radau M = 1: (W - dt nu A_h) u_1 = W (u_0 + dt f^E(u_0)) by dense algebra
    n = 8
    x, h = P.grid_p(n)
    u0 = 0.4 + np.abs(_rand((n, n), 7))
    dt, nu = 2e-3, 0.8
    cfg = SDCConfig(nu=nu, fe_kind=FE_BURGERS, node_kind=O.NODES_RADAU_RIGHT, M=1, inner="exact",
                    stencil=STENCIL_COMPACT4, bc=BC_PERIODIC)
    st = sdc_begin(u0, dt, h, cfg)
    sdc_sweep(st)
    W = _dense(lambda v: P.weight_p(v, h), n, 2)
    A = _dense(lambda v: P.laplacian_compact_p(v, h), n, 2)
    rhs = W @ (u0 + dt * P.burgers_advection(u0, h)).reshape(-1)
    ref = np.linalg.solve(W - dt * nu * A, rhs).reshape(n, n)
    assert np.max(np.abs(st.U[1] - ref)) < 1e-13
