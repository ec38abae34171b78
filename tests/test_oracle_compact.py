"""Pins for the oracle's fourth-order compact stencil and the compact sweep (eq. (5)).

Targets that do not reuse the oracle's own formulas: stencils written out as
point-by-point loops, the closed-form sine-mode eigenvalues, the O(h^4)
consistency of W^{-1} A_h, dense linear algebra for the implicit operator and
for one compact implicit Euler step, the modal collocation solution of the
compact heat problem, reduction to the second-order sweep when only f^E acts,
and the printed SDC sweep counts of Table 1(a).
"""

import csv
import os

import numpy as np
import pytest

import oracle as O
from oracle import compact as C
from oracle.sdc import SDCConfig, sdc_step, sdc_begin, sdc_sweep, sdc_residual, STENCIL_COMPACT4, PREC_MIXED

LOB, RAD = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(n):
    h = 1.0 / (n + 1)
    return (np.arange(n) + 1) * h, h


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def _at(u, *idx):
    """u at a multi-index, zero outside the grid (Dirichlet ghosts)."""
    n = u.shape[0]
    if any(i < 0 or i >= n for i in idx):
        return 0.0
    return u[idx]


def test_compact_laplacian_1d_is_three_point():
    u = _rand(15, 1)
    h = 1.0 / 16
    ref = np.array([(_at(u, i - 1) - 2 * u[i] + _at(u, i + 1)) / h ** 2 for i in range(15)])
    assert np.allclose(C.laplacian_compact(u, h), ref, rtol=0, atol=1e-9)


def test_compact_laplacian_2d_is_nine_point_loop():
    n, h = 9, 0.1
    u = _rand((n, n), 2)
    ref = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            edges = _at(u, i - 1, j) + _at(u, i + 1, j) + _at(u, i, j - 1) + _at(u, i, j + 1)
            corners = _at(u, i - 1, j - 1) + _at(u, i - 1, j + 1) + _at(u, i + 1, j - 1) + _at(u, i + 1, j + 1)
            ref[i, j] = (4 * edges + corners - 20 * u[i, j]) / (6 * h * h)
    assert np.max(np.abs(C.laplacian_compact(u, h) - ref)) < 1e-10


def test_compact_laplacian_3d_is_nineteen_point_loop():
    n, h = 5, 0.125
    u = _rand((n, n, n), 3)
    ref = np.zeros_like(u)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                faces = sum(_at(u, i + a, j + b, k + c) for a, b, c in
                            [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)])
                edges = sum(_at(u, i + a, j + b, k + c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                            if abs(a) + abs(b) + abs(c) == 2)
                ref[i, j, k] = (2 * faces + edges - 24 * u[i, j, k]) / (6 * h * h)
    assert np.max(np.abs(C.laplacian_compact(u, h) - ref)) < 1e-9


@pytest.mark.parametrize("d", [1, 2, 3])
def test_weight_is_the_compact_mass_stencil(d):
    n = {1: 11, 2: 7, 3: 5}[d]
    h = 1.0 / (n + 1)
    u = _rand((n,) * d, 4 + d)
    ref = np.zeros_like(u)
    for idx in np.ndindex(u.shape):
        nb = 0.0
        for ax in range(d):
            for s in (-1, 1):
                j = list(idx)
                j[ax] += s
                nb += _at(u, *j)
        centre = {1: 10.0, 2: 8.0, 3: 6.0}[d]
        ref[idx] = (centre * u[idx] + nb) / 12.0
    assert np.max(np.abs(C.weight(u, h) - ref)) < 1e-14


def test_eigenvalues_2d_closed_form():
    n = 15
    x, h = _grid(n)
    lam_a, lam_w = C.compact_eigenvalues(n, 2, h)
    for a, b in [(1, 1), (3, 7), (15, 15), (8, 2)]:
        mode = np.outer(np.sin(a * np.pi * x), np.sin(b * np.pi * x))
        th, ph = a * np.pi * h, b * np.pi * h
        la = (8 * np.cos(th) + 8 * np.cos(ph) + 4 * np.cos(th) * np.cos(ph) - 20) / (6 * h * h)
        lw = (8 + 2 * np.cos(th) + 2 * np.cos(ph)) / 12.0
        assert abs(lam_a[a - 1, b - 1] - la) < 1e-9 * abs(la)
        assert abs(lam_w[a - 1, b - 1] - lw) < 1e-14
        assert np.max(np.abs(C.laplacian_compact(mode, h) - la * mode)) < 1e-9 * abs(la)
        assert np.max(np.abs(C.weight(mode, h) - lw * mode)) < 1e-13


@pytest.mark.parametrize("d", [2, 3])
def test_fourth_order_consistency(d):
    # W^{-1} A_h u against the exact Laplacian of a smooth product of sines:
    # the error shrinks about 16-fold per halving of h (4-fold for L_h)
    errs, errs2 = [], []
    for n in ((15, 31, 63) if d == 2 else (7, 15, 31)):
        x, h = _grid(n)
        u = np.ones((n,) * d)
        for ax, k in zip(range(d), (1, 2, 1)):
            shape = [1] * d
            shape[ax] = n
            u = u * np.sin(k * np.pi * x).reshape(shape)
        exact = -(1 + 4 + (1 if d == 3 else 0)) * np.pi ** 2 * u
        errs.append(np.max(np.abs(C.solve_weight_exact(C.laplacian_compact(u, h), h) - exact)))
        errs2.append(np.max(np.abs(O.laplacian(u, h) - exact)))
    for k in range(len(errs) - 1):
        assert 14.0 < errs[k] / errs[k + 1] < 18.0
        assert 3.5 < errs2[k] / errs2[k + 1] < 4.5


def _dense(op, n, d):
    N = n ** d
    M = np.zeros((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = op(e.reshape((n,) * d)).reshape(N)
    return M


def test_exact_compact_solve_and_diagonal_against_dense():
    n, d = 7, 2
    h, c = 1.0 / 8, 0.013
    rhs = _rand((n, n), 7)
    B = _dense(lambda v: C.weight(v, h) - c * C.laplacian_compact(v, h), n, d)
    ref = np.linalg.solve(B, rhs.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(C.solve_compact_shifted_exact(rhs, c, h) - ref)) < 1e-12
    assert abs(C.compact_diagonal(d, c, h * h / 12, h) - B[0, 0]) < 1e-12
    assert np.allclose(B, B.T)  # W - c A_h is symmetric
    assert np.min(np.linalg.eigvalsh(B)) > 0


@pytest.mark.parametrize("c_h2", [0.5, 50.0])
def test_compact_vcycle_converges_and_iteration_matrix(c_h2):
    n = 31
    h = 1.0 / (n + 1)
    c = c_h2 * h * h
    rhs = _rand((n, n), 8)
    exact = C.solve_compact_shifted_exact(rhs, c, h)
    assert np.max(np.abs(C.vcycle_compact(exact, rhs, c, h, 3, 3) - exact)) < 1e-12  # fixed point
    u = np.zeros_like(rhs)
    errs = []
    for _ in range(8):
        u = C.vcycle_compact(u, rhs, c, h, 3, 3)
        errs.append(np.max(np.abs(u - exact)))
    assert errs[-1] < 1e-8 * np.max(np.abs(exact))
    assert errs[3] / errs[2] < 0.15
    # spectral radius of the explicitly formed iteration matrix on a small grid
    n2, h2 = 7, 1.0 / 8
    c2 = c_h2 * h2 * h2
    zero = np.zeros((n2, n2))
    G = _dense(lambda e0: C.vcycle_compact(e0, zero, c2, h2, 3, 3), n2, 2)
    assert max(abs(np.linalg.eigvals(G))) < 0.2


def test_first_compact_sweep_is_compact_implicit_euler():
    # right Radau M = 1: one sweep from the spread iterate solves
    # (W - dt nu A_h) u_1 = W u_0 (eq. (5) with S F~(u^0) = dt nu A_h u_0)
    n, d = 7, 2
    x, h = _grid(n)
    u0 = _rand((n, n), 9)
    dt, nu = 0.01, 1.3
    cfg = SDCConfig(nu=nu, node_kind=RAD, M=1, inner="exact", stencil=STENCIL_COMPACT4)
    st = sdc_begin(u0, dt, h, cfg)
    sdc_sweep(st)
    W = _dense(lambda v: C.weight(v, h), n, d)
    A = _dense(lambda v: C.laplacian_compact(v, h), n, d)
    ref = np.linalg.solve(W - dt * nu * A, W @ u0.reshape(-1)).reshape(n, n)
    assert np.max(np.abs(st.U[1] - ref)) < 1e-13


def _compact_collocation(u0, dt, nu, h, kind, M):
    from scipy.fft import dstn, idstn
    lam_a, lam_w = C.compact_eigenvalues(u0.shape[0], u0.ndim, h)
    R = O.stability_function(dt * nu * lam_a / lam_w, kind, M)
    return idstn(dstn(u0, type=1, norm="ortho") * R, type=1, norm="ortho")


@pytest.mark.parametrize("inner,kind,M,prec", [("exact", LOB, 5, 0), ("mg", LOB, 3, 0), ("mg", RAD, 3, 0),
                                                ("mg", LOB, 5, PREC_MIXED), ("exact", O.NODES_LEGENDRE, 3, 0),
                                                ("mg", O.NODES_LEGENDRE, 2, 0)])
def test_compact_sdc_converges_to_compact_collocation(inner, kind, M, prec):
    n = 31
    x, h = _grid(n)
    u0 = np.outer(np.sin(np.pi * x), np.sin(2 * np.pi * x)) + 0.3 * np.outer(np.sin(5 * np.pi * x), np.sin(np.pi * x))
    dt, nu = 2e-3, 1.0
    coll = _compact_collocation(u0, dt, nu, h, kind, M)
    cfg = SDCConfig(nu=nu, node_kind=kind, M=M, inner=inner, smoother=1, nu1=3, nu2=3, precision=prec,
                    stencil=STENCIL_COMPACT4, tol=1e-12 if prec == 0 else 1e-10, max_sweeps=200)
    u, st = sdc_step(u0, dt, h, cfg)
    assert st.status == "ok"
    tol = 1e-11 if prec == 0 else 1e-8
    assert np.linalg.norm(u - coll) / np.linalg.norm(coll) < tol
    # the compact collocation solution differs from the second-order one by the spatial error
    coll2 = O.collocation_heat_modal(u0, dt, nu, h, kind, M)
    assert np.linalg.norm(coll - coll2) / np.linalg.norm(coll) > 1e-6


def test_compact_residual_inverts_w_once_per_node():
    # residual of an arbitrary iterate against dense algebra:
    # max_m |u_0 + dt (Q kron W^{-1})(W f^E + nu A_h) U - u_m|
    n, M = 7, 3
    x, h = _grid(n)
    u0 = _rand((n, n), 10)
    cfg = SDCConfig(nu=0.7, fe_kind=O.FE_CUBIC, node_kind=LOB, M=M, stencil=STENCIL_COMPACT4)
    st = sdc_begin(u0, 0.05, h, cfg)
    rng = np.random.default_rng(11)
    for j in range(1, M + 1):
        st.U[j] = u0 + 0.01 * rng.standard_normal(u0.shape)
        st.F[j] = C.weight(O.f_explicit(st.U[j], O.FE_CUBIC), h) + 0.7 * C.laplacian_compact(st.U[j], h)
    W = _dense(lambda v: C.weight(v, h), n, 2)
    A = _dense(lambda v: C.laplacian_compact(v, h), n, 2)
    Q = O.qmatrix(LOB, M)
    f = [np.linalg.solve(W, W @ O.f_explicit(st.U[j], O.FE_CUBIC).reshape(-1) + 0.7 * A @ st.U[j].reshape(-1))
         for j in range(1, M + 1)]
    ref = max(np.max(np.abs(u0.reshape(-1) + 0.05 * sum(Q[m, j] * f[j] for j in range(M)) - st.U[m + 1].reshape(-1)))
              for m in range(M))
    assert abs(sdc_residual(st) - ref) < 1e-12 * max(1.0, ref)


def test_compact_with_explicit_part_only_equals_second_order_sweep():
    # nu = 0: W cancels from eq. (5) and from the residual, leaving eq. (4)
    n = 15
    x, h = _grid(n)
    u0 = 1.5 * np.outer(np.sin(np.pi * x), np.sin(3 * np.pi * x))
    base = dict(nu=0.0, fe_kind=O.FE_CUBIC, node_kind=LOB, M=3, inner="exact", tol=1e-13, max_sweeps=60)
    u2, s2 = sdc_step(u0, 0.05, h, SDCConfig(**base))
    uc, sc = sdc_step(u0, 0.05, h, SDCConfig(stencil=STENCIL_COMPACT4, **base))
    assert s2.sweeps == sc.sweeps
    assert np.max(np.abs(uc - u2)) < 1e-12


def test_compact_exact_sdc_reproduces_table1_sdc_sweeps():
    # the paper's own stencil: sweep counts with (near-)exact solves match the
    # printed SDC column of Table 1(a) except nu = 1, M = 3 (3 here, 4 printed)
    rows = {}
    with open(os.path.join(GOLDEN, "table1.csv")) as fh:
        for r in csv.DictReader(line for line in fh if not line.startswith("#")):
            if r["problem"] == "heat":
                rows[(float(r["nu"]), int(r["M"]))] = int(r["sdc_sweeps"])
    n = 63
    x, h = _grid(n)
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    got = {}
    for (nu, M) in rows:
        cfg = SDCConfig(nu=nu, node_kind=LOB, M=M, inner="exact", tol=5e-8, stencil=STENCIL_COMPACT4)
        _, st = sdc_step(u0, 1e-3, h, cfg)
        got[(nu, M)] = st.sweeps
    assert [k for k in rows if got[k] != rows[k]] == [(1.0, 3)]
