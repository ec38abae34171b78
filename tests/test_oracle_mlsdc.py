"""Pins for the oracle's two-level MLSDC (Sec. 5): its fixed point is the fine
collocation solution, the FAS term makes the restricted fine solution a fixed
point of the coarse sweep, and without coarsening an iteration is two plain
sweeps."""

import numpy as np
import pytest

import oracle as O
from oracle.mlsdc import mlsdc_step, inject, fas_term, _coarse_state, mlsdc_iteration, MLSDCStats, prolong_cubic
from oracle.sdc import SDCConfig, sdc_begin, sdc_sweep, sdc_step

LOB, RAD, LEG = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT, O.NODES_LEGENDRE


def _smooth_u0(n, d, seed, K=6):
    rng = np.random.default_rng(seed)
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    u = np.zeros((n,) * d)
    for _ in range(K):
        a = rng.integers(1, 6, size=d)
        t = rng.standard_normal() / float(np.sum(a * a))
        for ax in range(d):
            shape = [1] * d
            shape[ax] = n
            t = t * np.sin(a[ax] * np.pi * x).reshape(shape)
        u = u + t
    return u, h


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_injection_picks_odd_points():
    u = np.arange(7 * 7, dtype=float).reshape(7, 7)
    c = inject(u)
    assert c.shape == (3, 3)
    for I in range(3):
        for J in range(3):
            assert c[I, J] == u[2 * I + 1, 2 * J + 1]


@pytest.mark.parametrize("d,n,kind,M,inner", [(1, 63, LOB, 3, "exact"), (2, 31, LOB, 5, "exact"),
                                              (2, 31, RAD, 3, "exact"), (1, 63, LEG, 3, "exact"),
                                              (2, 31, LOB, 3, "mg")])
def test_mlsdc_converges_to_fine_collocation(d, n, kind, M, inner):
    u0, h = _smooth_u0(n, d, 41)
    dt, nu = 5e-3, 1.0
    cfg = SDCConfig(nu=nu, node_kind=kind, M=M, inner=inner, tol=1e-13, max_sweeps=100)
    u, st, _ = mlsdc_step(u0, dt, h, cfg)
    assert st.status == "ok"
    assert _rel(u, O.collocation_heat_modal(u0, dt, nu, h, kind, M)) < 1e-11


def test_mlsdc_cubic_reaches_newton_collocation():
    u0, h = _smooth_u0(7, 2, 42)
    u0 = 3.0 * u0
    cfg = SDCConfig(nu=0.2, fe_kind=O.FE_CUBIC, node_kind=LOB, M=3, inner="exact", tol=1e-13)
    u, st, _ = mlsdc_step(u0, 0.05, h, cfg)
    assert st.status == "ok"
    assert _rel(u, O.collocation_dense(u0, 0.05, 0.2, h, O.FE_CUBIC, LOB, 3)) < 1e-11


def test_fas_makes_restricted_solution_a_coarse_fixed_point():
    # at the fine collocation solution U*, R U* solves the coarse FAS problem:
    # one coarse sweep (exact solves) from R U* leaves it unchanged
    n, d = 31, 2
    u0, h = _smooth_u0(n, d, 43)
    u0 = 2.0 * u0
    cfg = SDCConfig(nu=0.7, fe_kind=O.FE_CUBIC, node_kind=LOB, M=3, inner="exact")
    fine = sdc_begin(u0, 4e-3, h, cfg)
    for _ in range(40):
        sdc_sweep(fine)
    assert fine.stats.residual < 1e-14
    coarse, R = _coarse_state(fine, True)
    RU = [u.copy() for u in coarse.U]
    tau = fas_term(fine, coarse, R)
    assert max(np.max(np.abs(t)) for t in tau[2:]) > 1e-6  # the term is not trivially zero
    sdc_sweep(coarse, fas=tau)
    for m in range(1, cfg.M + 1):
        assert np.max(np.abs(coarse.U[m] - RU[m])) < 1e-13
    # with the FAS term left out the coarse sweep moves away from R U*
    coarse2, _ = _coarse_state(fine, True)
    sdc_sweep(coarse2)
    assert max(np.max(np.abs(coarse2.U[m] - RU[m])) for m in range(1, cfg.M + 1)) > 1e-6


def test_without_coarsening_an_iteration_is_two_sweeps():
    n, d = 31, 2
    u0, h = _smooth_u0(n, d, 44)
    cfg = SDCConfig(nu=1.0, fe_kind=O.FE_CUBIC, node_kind=RAD, M=3, inner="mg", vcycles=2)
    fine = sdc_begin(u0, 5e-3, h, cfg)
    stats = MLSDCStats()
    ref = sdc_begin(u0, 5e-3, h, cfg)
    for _ in range(3):
        mlsdc_iteration(fine, stats, coarsen=False)
        sdc_sweep(ref)
        sdc_sweep(ref)
        for m in range(1, cfg.M + 1):
            assert np.max(np.abs(fine.U[m] - ref.U[m])) < 1e-14
    assert stats.vcycles == stats.coarse_vcycles == 3 * 3 * 2


def test_cubic_interpolation_exact_for_cubics_vanishing_at_the_boundary():
    # per axis the known values are the coarse points and the zero boundary
    # values, so x (1 - x)(a + b x) (degree 3) is reproduced exactly
    n = 15
    x = np.arange(1, n + 1) / (n + 1)
    p = lambda t: t * (1 - t) * (0.3 - 1.7 * t)  # noqa: E731
    q = lambda t: t * (1 - t) * (2.0 + 0.5 * t)  # noqa: E731
    np.testing.assert_allclose(prolong_cubic(p(x[1::2])), p(x), atol=1e-15)
    fine2 = np.outer(p(x), q(x))
    np.testing.assert_allclose(prolong_cubic(fine2[1::2, 1::2]), fine2, atol=1e-15)
    fine3 = np.einsum("i,j,k->ijk", q(x), p(x), q(x))
    np.testing.assert_allclose(prolong_cubic(fine3[1::2, 1::2, 1::2]), fine3, atol=1e-15)
    # and the coarse points keep their values
    c = np.random.default_rng(3).standard_normal((7, 7))
    assert np.array_equal(prolong_cubic(c)[1::2, 1::2], c)


def test_cubic_interpolation_fourth_order():
    errs = []
    for nc in (15, 31, 63):
        n = 2 * nc + 1
        x = np.arange(1, n + 1) / (n + 1)
        f = np.sin(np.pi * x) * np.exp(x)
        errs.append(np.max(np.abs(prolong_cubic(f[1::2]) - f)))
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_mlsdc_needs_fewer_fine_sweeps_than_sdc_when_coarse_level_resolves():
    # well resolved and mildly stiff (nu dt / h^2 = 0.8): the coarse sweep does
    # part of the work, so fewer fine sweeps reach the tolerance
    n, d = 127, 2
    u0, h = _smooth_u0(n, d, 45)
    cfg = SDCConfig(nu=0.1, node_kind=LOB, M=5, inner="exact", tol=1e-10)
    _, sst = sdc_step(u0, 1e-3, h, cfg)
    _, mst, _ = mlsdc_step(u0, 1e-3, h, cfg)
    assert sst.status == "ok" and mst.status == "ok"
    assert mst.iterations < sst.sweeps
