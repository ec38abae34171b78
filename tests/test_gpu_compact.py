"""GPU parity of the fourth-order compact stencil (Sec. 3, eq. (5)) against the oracle.

Components and V-cycles of B_H = I + (h^2/12) L_H - c A_H (weighted Jacobi,
omega = 1), whole compact ISDC steps (heat and reaction-diffusion, Lobatto
and right Radau, FP64 and float32 V-cycles, classical and early-exit modes)
and the Table 1(a) replay with the paper's own stencil.  The GPU inverts W
for the residual with warm-started V-cycles and the oracle exactly; sweep
counts must still coincide, and states after equal sweeps agree to 1e-12.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import compact as C
from oracle.sdc import SDCConfig, sdc_step, sdc_begin, sdc_sweep, STENCIL_COMPACT4
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, host, rel_l2, require_gpu, random_field

pytestmark = pytest.mark.gpu

LOB, RAD = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _plan(n, nu=1.0, fe=O.FE_ZERO, **par):
    from paper_1401_7824_amd import Plan, STENCIL_COMPACT4 as SC
    par.setdefault("smoother", 1)
    par.setdefault("nu_pre", 3)
    par.setdefault("nu_post", 3)
    return Plan(2, n, nu, fe, stencil=SC, **par)


def _np(tdt):
    return np.float64 if tdt == torch.float64 else np.float32


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("level", [0, 1])
def test_compact_components(level, dtype):
    from paper_1401_7824_amd import OP_SMOOTH, OP_RESTRICT, OP_RESIDUAL_NORM
    n0 = 255
    announce("compact components", level, dtype)
    p = _plan(n0)
    h = 1.0 / (n0 + 1)
    w = h * h / 12.0
    n, H = (n0 - 1) // 2 if level else n0, 2 * h if level else h
    c = 0.3 * 1e-3
    nd = _np(dtype)
    rhs = random_field((n, n), 1).astype(nd)
    u = random_field((n, n), 2).astype(nd)
    prec = 0 if dtype == torch.float64 else 1
    out = torch.empty((n, n), dtype=dtype, device="cuda")
    p.mg_op(OP_SMOOTH, level, c, a=dev(rhs, dtype), b=dev(u, dtype), out=out)
    ref = C.smooth_compact(u, rhs, c, w, H, 1.0)
    assert rel_l2(host(out), ref) < TOL[dtype]
    nc = (n - 1) // 2
    rc = torch.empty((nc, nc), dtype=dtype, device="cuda")
    p.mg_op(OP_RESTRICT, level, c, a=dev(rhs, dtype), b=dev(u, dtype), out=rc)
    ref = O.restrict_fw(rhs - C.apply_compact_shifted(u, c, H, w))
    assert rel_l2(host(rc), ref) < TOL[dtype]
    res = p.mg_op(OP_RESIDUAL_NORM, level, c, a=dev(rhs, dtype), b=dev(u, dtype))
    ref = float(np.max(np.abs(rhs - C.apply_compact_shifted(u, c, H, w))))
    assert abs(res - ref) < (1e-12 if prec == 0 else 1e-4) * ref


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_compact_coarse_tail(dtype):
    from paper_1401_7824_amd import OP_COARSE
    n0 = 255
    announce("compact tail", dtype)
    p = _plan(n0, nu_pre=2, nu_post=1)
    h = 1.0 / (n0 + 1)
    level, n, H = 2, 63, 4 * h
    c = 5e-3
    nd = _np(dtype)
    rhs = random_field((n, n), 3).astype(nd)
    out = torch.empty((n, n), dtype=dtype, device="cuda")
    p.mg_op(OP_COARSE, level, c, a=dev(rhs, dtype), out=out)
    ref = C.vcycle_compact(np.zeros((n, n), nd), rhs, c, H, 2, 1, 1.0, w=h * h / 12.0)
    assert rel_l2(host(out), ref) < TOL[dtype] * 10


@pytest.mark.parametrize("n", [63, 255, 511])
def test_compact_vcycle(n):
    announce("compact vcycle", n)
    p = _plan(n)
    h = 1.0 / (n + 1)
    c = 1e-3 * 0.37
    rhs = random_field((n, n), 4)
    u0 = 0.1 * random_field((n, n), 5)
    u = dev(u0)
    res = p.vcycle(c, dev(rhs), u, 2, want_residual=True)
    ref = u0
    for _ in range(2):
        ref = C.vcycle_compact(ref, rhs, c, h, 3, 3, 1.0)
    assert rel_l2(host(u), ref) < 1e-12
    assert abs(res - C.residual_compact_inf(ref, rhs, c, h)) < 1e-9 * max(res, 1e-30) + 1e-14


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nus", [(1, 1), (2, 2), (4, 5), (0, 2), (2, 0)])
def test_compact_vcycle_smoothing_counts(nus, dtype):
    # every split of the smoothing steps over the launches of a level: up to
    # three steps fused with the restriction / prolongation, the rest three
    # per launch, none at all (plain restriction / prolongation)
    n, (nu1, nu2) = 255, nus
    announce("compact vcycle nu", nus, dtype)
    p = _plan(n, nu_pre=nu1, nu_post=nu2)
    h = 1.0 / (n + 1)
    c = 1e-3 * 0.37
    nd = _np(dtype)
    rhs = random_field((n, n), 41).astype(nd)
    u0 = (0.1 * random_field((n, n), 42)).astype(nd)
    u = dev(u0, dtype)
    p.vcycle(c, dev(rhs, dtype), u, 2)
    ref = u0
    for _ in range(2):
        ref = C.vcycle_compact(ref, rhs, c, h, nu1, nu2, 1.0)
    assert rel_l2(host(u), ref) < (1e-12 if dtype == torch.float64 else 2e-5)


def _cfg(nu, fe, kind, M, prec=0, **kw):
    base = dict(nu=nu, fe_kind=fe, node_kind=kind, M=M, inner="mg", smoother=1, nu1=3, nu2=3, precision=prec,
                stencil=STENCIL_COMPACT4)
    base.update(kw)
    return SDCConfig(**base)


def _par(kind, M, prec=0, **kw):
    d = dict(node_kind=kind, M=M, precision=prec, smoother=1, nu_pre=3, nu_post=3)
    d.update(kw)
    return d


@pytest.mark.parametrize("case", [
    ("heat-lob3", 255, 1.0, O.FE_ZERO, LOB, 3, 2e-3),
    ("rd-lob5", 127, 0.1, O.FE_CUBIC, LOB, 5, 1e-3),
    ("heat-rad3", 255, 0.5, O.FE_ZERO, RAD, 3, 2e-3),
], ids=lambda c: c[0])
def test_compact_fixed_sweeps_equal_oracle(case):
    name, n, nu, fe, kind, M, dt = case
    announce("compact sweeps", name)
    h = 1.0 / (n + 1)
    u0 = 2.0 * W.sine_field(n, 2, W.draw_modes(2, 8, seed=21))
    p = _plan(n, nu, fe, **_par(kind, M))
    u = dev(u0)
    p.begin(u, dt)
    st = sdc_begin(u0, dt, h, _cfg(nu, fe, kind, M))
    for k in range(3):
        rg = p.sweep()
        ro = sdc_sweep(st)
        assert abs(rg - ro) <= 1e-5 * ro + 1e-15, (k, rg, ro)  # W^{-1} by warm-started V-cycles vs exactly
        for j in range(1, M + 1):
            got = host(p.node_values(j))
            assert rel_l2(got, st.U[j]) < 1e-12, (k, j)
    p.end(u)


@pytest.mark.parametrize("case", [
    ("heat-lob3", 255, 1.0, O.FE_ZERO, LOB, 3, 2e-3, 1e-10),
    ("rd-lob5", 255, 0.1, O.FE_CUBIC, LOB, 5, 1e-3, 1e-10),
    ("heat-rad5", 127, 2.0, O.FE_ZERO, RAD, 5, 1e-3, 1e-9),
], ids=lambda c: c[0])
def test_compact_step_equals_oracle(case):
    name, n, nu, fe, kind, M, dt, tol = case
    announce("compact step", name)
    h = 1.0 / (n + 1)
    u0 = 2.0 * W.sine_field(n, 2, W.draw_modes(2, 8, seed=22))
    p = _plan(n, nu, fe, **_par(kind, M, sdc_tol=tol))
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst = sdc_step(u0, dt, h, _cfg(nu, fe, kind, M, tol=tol))
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert rel_l2(host(u), ref) < 1e-12


def test_compact_mixed_precision_reaches_collocation():
    from scipy.fft import dstn, idstn
    announce("compact mixed")
    n, nu, dt, M = 255, 1.0, 2e-3, 5
    h = 1.0 / (n + 1)
    u0 = W.sine_field(n, 2, W.draw_modes(2, 8, seed=23))
    lam_a, lam_w = C.compact_eigenvalues(n, 2, h)
    R = O.stability_function(dt * nu * lam_a / lam_w, LOB, M)
    coll = idstn(dstn(u0, type=1, norm="ortho") * R, type=1, norm="ortho")
    p = _plan(n, nu, **_par(LOB, M, prec=1, sdc_tol=1e-11))
    u = dev(u0)
    st = p.step(u, dt)
    assert st.status == "ok"
    assert rel_l2(host(u), coll) < 1e-8


@pytest.mark.parametrize("mode", ["classical", "early"])
def test_compact_inner_modes_equal_oracle(mode):
    announce("compact inner mode", mode)
    n, nu, dt, M = 127, 10.0, 1e-3, 3
    h = 1.0 / (n + 1)
    u0 = W.sine_field(n, 2, W.draw_modes(2, 6, seed=24))
    kw = dict(vcycles=0) if mode == "classical" else dict(vcycles=2, early_exit=True)
    p = _plan(n, nu, **_par(LOB, M, sdc_tol=1e-9, inner_tol=1e-9, **kw))
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst = sdc_step(u0, dt, h, _cfg(nu, O.FE_ZERO, LOB, M, tol=1e-9, inner_tol=1e-9,
                                        early_exit=(mode == "early"), vcycles=kw["vcycles"]))
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert rel_l2(host(u), ref) < 1e-12


ROWS = [(nu, M) for nu in (1.0, 10.0, 100.0) for M in (3, 5, 7)]


@pytest.mark.parametrize("isdc", [False, True], ids=["sdc", "isdc"])
@pytest.mark.parametrize("nu,M", ROWS)
def test_compact_table1_counts_equal_oracle(nu, M, isdc):
    announce("compact table1", nu, M, isdc)
    n, dt = 63, 1e-3
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) * h
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    mode = dict(vcycles=2, early_exit=True) if isdc else dict(vcycles=0)
    p = _plan(n, nu, **_par(LOB, M, sdc_tol=5e-8, inner_tol=1e-9, max_sweeps=100, **mode))
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst = sdc_step(u0, dt, h, _cfg(nu, O.FE_ZERO, LOB, M, tol=5e-8, inner_tol=1e-9, max_sweeps=100,
                                        early_exit=isdc, vcycles=mode["vcycles"]))
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert rel_l2(host(u), ref) < 1e-12


def test_compact_unsupported_combinations():
    from paper_1401_7824_amd import Plan, Batch, ISDCError, STENCIL_COMPACT4 as SC, KERNEL_TAIL, KERNEL_SMOOTH_RESTRICT
    announce("compact unsupported")
    with pytest.raises(ISDCError):
        Plan(3, 15, 1.0, stencil=SC, smoother=1)
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, stencil=SC, smoother=0)
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, stencil=SC, smoother=1, guess=1)
    p = Plan(2, 31, 1.0, stencil=SC, smoother=1)
    with pytest.raises(ISDCError):
        p.time_kernel(KERNEL_SMOOTH_RESTRICT, 0, 1e-3, 0, 1)
    us, nbytes = p.time_kernel(KERNEL_TAIL, 0, 1e-3, 0, 2)
    assert us > 0 and nbytes == 2 * 31 * 31 * 8
    b = Batch(2, 2)
    u = dev(np.zeros((31, 31)))
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, stencil=SC, smoother=1)
