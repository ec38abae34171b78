"""GPU parity of the periodic compact stencil and the WENO5 viscous Burgers
setup (Sec. 4.1, Table 1(b)) against the oracle.

Components and V-cycles of B_H = I + (h^2/12) L_H - c A_H on periodic grids
(coarse point I on fine point 2I, weighted Jacobi with omega = 1), the WENO5
advection f^E, fixed sweeps and whole steps of Burgers and periodic heat, and
the Table 1(b) replay: classical SDC and ISDC V-cycle and sweep counts must
equal the oracle's.  The GPU inverts W for the residual with warm-started
V-cycles and the oracle with the FFT, so residuals agree to 1e-5 relative and
states after equal sweeps to 1e-12.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import periodic as P
from oracle.sdc import SDCConfig, sdc_step, sdc_begin, sdc_sweep, STENCIL_COMPACT4, BC_PERIODIC, FE_BURGERS
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, host, rel_l2, require_gpu, random_field

pytestmark = pytest.mark.gpu

LOB, RAD = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _plan(n, nu=1.0, fe=O.FE_ZERO, **par):
    from paper_1401_7824_amd import Plan, STENCIL_COMPACT4 as SC, BC_PERIODIC as BP
    par.setdefault("smoother", 1)
    par.setdefault("nu_pre", 3)
    par.setdefault("nu_post", 3)
    return Plan(2, n, nu, fe, stencil=SC, bc=BP, **par)


def _np(tdt):
    return np.float64 if tdt == torch.float64 else np.float32


def _smooth_ref(u, rhs, c, H, w):
    b0 = P.compact_diagonal_p(2, c, w, H)
    return u + (rhs - P.apply_compact_shifted_p(u, c, H, w)) / u.dtype.type(b0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("level", [0, 1, 3])
def test_periodic_components(level, dtype):
    from paper_1401_7824_amd import OP_SMOOTH, OP_RESTRICT, OP_PROLONG, OP_RESIDUAL_NORM
    n0 = 256
    announce("periodic components", level, dtype)
    p = _plan(n0)
    h = 2.0 / n0
    w = h * h / 12.0
    n, H = n0 >> level, h * 2 ** level
    c = 0.3 * 1e-3
    nd = _np(dtype)
    rhs = random_field((n, n), 11).astype(nd)
    u = random_field((n, n), 12).astype(nd)
    out = torch.empty((n, n), dtype=dtype, device="cuda")
    p.mg_op(OP_SMOOTH, level, c, a=dev(rhs, dtype), b=dev(u, dtype), out=out)
    assert rel_l2(host(out), _smooth_ref(u, rhs, c, H, w)) < TOL[dtype]
    nc = n // 2
    rc = torch.empty((nc, nc), dtype=dtype, device="cuda")
    p.mg_op(OP_RESTRICT, level, c, a=dev(rhs, dtype), b=dev(u, dtype), out=rc)
    assert rel_l2(host(rc), P.restrict_fw_p(rhs - P.apply_compact_shifted_p(u, c, H, w))) < TOL[dtype]
    ec = random_field((nc, nc), 13).astype(nd)
    ud = dev(u, dtype)
    p.mg_op(OP_PROLONG, level, c, a=dev(ec, dtype), out=ud)
    assert rel_l2(host(ud), u + P.prolong_linear_p(ec)) < TOL[dtype]
    res = p.mg_op(OP_RESIDUAL_NORM, level, c, a=dev(rhs, dtype), b=dev(u, dtype))
    ref = float(np.max(np.abs(rhs - P.apply_compact_shifted_p(u, c, H, w))))
    assert abs(res - ref) < (1e-12 if dtype == torch.float64 else 1e-4) * ref


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n0,level", [(128, 2), (16, 0), (128, 4), (4, 0)])
def test_periodic_coarse_tail(n0, level, dtype):
    from paper_1401_7824_amd import OP_COARSE
    announce("periodic tail", n0, level, dtype)
    p = _plan(n0, nu_pre=2, nu_post=1)
    h = 2.0 / n0
    n, H = n0 >> level, h * 2 ** level
    c = 5e-3
    nd = _np(dtype)
    rhs = random_field((n, n), 14).astype(nd)
    out = torch.empty((n, n), dtype=dtype, device="cuda")
    p.mg_op(OP_COARSE, level, c, a=dev(rhs, dtype), out=out)
    ref = P.vcycle_compact_p(np.zeros((n, n), nd), rhs, c, H, 2, 1, 1.0, w=h * h / 12.0)
    assert rel_l2(host(out), ref) < TOL[dtype] * 10


@pytest.mark.parametrize("n", [8, 64, 256, 512])
def test_periodic_vcycle(n):
    announce("periodic vcycle", n)
    p = _plan(n)
    h = 2.0 / n
    c = 1e-3 * 0.37
    rhs = random_field((n, n), 15)
    u0 = 0.1 * random_field((n, n), 16)
    u = dev(u0)
    res = p.vcycle(c, dev(rhs), u, 2, want_residual=True)
    ref = u0
    for _ in range(2):
        ref = P.vcycle_compact_p(ref, rhs, c, h, 3, 3, 1.0)
    assert rel_l2(host(u), ref) < 1e-12
    assert abs(res - P.residual_compact_inf_p(ref, rhs, c, h)) < 1e-9 * max(res, 1e-30) + 1e-14


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nus", [(1, 1), (2, 2), (4, 5), (0, 2), (2, 0)])
def test_periodic_vcycle_smoothing_counts(nus, dtype):
    # the launches of a periodic level for every split of the smoothing steps
    n, (nu1, nu2) = 256, nus
    announce("periodic vcycle nu", nus, dtype)
    p = _plan(n, nu_pre=nu1, nu_post=nu2)
    h = 2.0 / n
    c = 1e-3 * 0.37
    nd = _np(dtype)
    rhs = random_field((n, n), 43).astype(nd)
    u0 = (0.1 * random_field((n, n), 44)).astype(nd)
    u = dev(u0, dtype)
    p.vcycle(c, dev(rhs, dtype), u, 2)
    ref = u0
    for _ in range(2):
        ref = P.vcycle_compact_p(ref, rhs, c, h, nu1, nu2, 1.0)
    assert rel_l2(host(u), ref) < (1e-12 if dtype == torch.float64 else 2e-5)


@pytest.mark.parametrize("n", [4, 8, 128, 1024])
def test_weno_burgers_advection(n):
    from paper_1401_7824_amd import OP_EXPLICIT
    announce("weno advection", n)
    p = _plan(n, 1.0, FE_BURGERS)
    h = 2.0 / n
    for u0 in (W.gaussian_periodic(n, 0.1), 0.5 + W.periodic_field(n, 17), random_field((n, n), 18)):
        out = torch.empty((n, n), dtype=torch.float64, device="cuda")
        p.mg_op(OP_EXPLICIT, 0, 0.0, a=dev(u0), out=out)
        ref = P.burgers_advection(u0, h)
        assert rel_l2(host(out), ref) < 1e-13


def _cfg(nu, fe, kind, M, prec=0, **kw):
    base = dict(nu=nu, fe_kind=fe, node_kind=kind, M=M, inner="mg", smoother=1, nu1=3, nu2=3, precision=prec,
                stencil=STENCIL_COMPACT4, bc=BC_PERIODIC)
    base.update(kw)
    return SDCConfig(**base)


def _par(kind, M, prec=0, **kw):
    d = dict(node_kind=kind, M=M, precision=prec, smoother=1, nu_pre=3, nu_post=3)
    d.update(kw)
    return d


@pytest.mark.parametrize("case", [
    ("burgers-nu0.1-lob3", 128, 0.1, FE_BURGERS, LOB, 3, 1e-3, 0),
    ("burgers-nu10-lob5", 128, 10.0, FE_BURGERS, LOB, 5, 1e-3, 0),
    ("burgers-nu1-rad3", 64, 1.0, FE_BURGERS, RAD, 3, 2e-3, 0),
    ("burgers-nu1-lob3-mixed", 128, 1.0, FE_BURGERS, LOB, 3, 1e-3, 1),
    ("heat-lob3", 256, 1.0, O.FE_ZERO, LOB, 3, 2e-3, 0),
    ("cubic-rad5", 32, 0.2, O.FE_CUBIC, RAD, 5, 1e-3, 0),
], ids=lambda c: c[0])
def test_periodic_fixed_sweeps_equal_oracle(case):
    name, n, nu, fe, kind, M, dt, prec = case
    announce("periodic sweeps", name)
    h = 2.0 / n
    u0 = W.gaussian_periodic(n, 0.1) if fe == FE_BURGERS else W.periodic_field(n, 19)
    p = _plan(n, nu, fe, **_par(kind, M, prec))
    u = dev(u0)
    p.begin(u, dt)
    st = sdc_begin(u0, dt, h, _cfg(nu, fe, kind, M, prec))
    state_tol, res_tol = (1e-12, 1e-5) if prec == 0 else (1e-6, 1e-2)
    for k in range(3):
        rg = p.sweep()
        ro = sdc_sweep(st)
        assert abs(rg - ro) <= res_tol * ro + 1e-15, (k, rg, ro)  # W^{-1} by warm-started V-cycles vs FFT
        for j in range(1, M + 1):
            assert rel_l2(host(p.node_values(j)), st.U[j]) < state_tol, (k, j)
    p.end(u)


@pytest.mark.parametrize("case", [
    ("burgers-nu1-lob5", 128, 1.0, FE_BURGERS, LOB, 5, 1e-3, 1e-10),
    ("burgers-nu10-rad3", 64, 10.0, FE_BURGERS, RAD, 3, 1e-3, 1e-10),
    ("heat-lob3", 128, 2.0, O.FE_ZERO, LOB, 3, 1e-3, 1e-11),
], ids=lambda c: c[0])
def test_periodic_step_equals_oracle(case):
    name, n, nu, fe, kind, M, dt, tol = case
    announce("periodic step", name)
    h = 2.0 / n
    u0 = W.gaussian_periodic(n, 0.1) if fe == FE_BURGERS else W.periodic_field(n, 20)
    p = _plan(n, nu, fe, **_par(kind, M, sdc_tol=tol))
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst = sdc_step(u0, dt, h, _cfg(nu, fe, kind, M, tol=tol))
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert rel_l2(host(u), ref) < 1e-12


def test_periodic_mixed_precision_reaches_collocation():
    announce("periodic mixed")
    n, nu, dt, M = 256, 1.0, 2e-3, 5
    h = 2.0 / n
    u0 = W.periodic_field(n, 21)
    _, lam_a, lam_w = P.eigenvalues_p(n, 2, h)
    R = O.stability_function(dt * nu * lam_a / lam_w, LOB, M)
    coll = np.real(np.fft.ifftn(np.fft.fftn(u0) * R))
    p = _plan(n, nu, **_par(LOB, M, prec=1, sdc_tol=1e-11))
    u = dev(u0)
    st = p.step(u, dt)
    assert st.status == "ok"
    assert rel_l2(host(u), coll) < 1e-8


ROWS = [(nu, M) for nu in (0.1, 1.0, 10.0) for M in (3, 5, 7)]


@pytest.mark.parametrize("isdc", [False, True], ids=["sdc", "isdc"])
@pytest.mark.parametrize("nu,M", ROWS)
def test_burgers_table1b_counts_equal_oracle(nu, M, isdc):
    # Table 1(b) setup: n = 128 (h = 1/64), Gaussian sigma = 0.1, dt = 1e-3,
    # Gauss-Lobatto, SDC residual < 5e-8; classical SDC cycles to 1e-9, ISDC L = 2
    announce("burgers table1b", nu, M, isdc)
    n, dt = 128, 1e-3
    h = 2.0 / n
    u0 = W.gaussian_periodic(n, 0.1)
    mode = dict(vcycles=2, early_exit=True) if isdc else dict(vcycles=0)
    p = _plan(n, nu, FE_BURGERS, **_par(LOB, M, sdc_tol=5e-8, inner_tol=1e-9, max_sweeps=100, **mode))
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst = sdc_step(u0, dt, h, _cfg(nu, FE_BURGERS, LOB, M, tol=5e-8, inner_tol=1e-9, max_sweeps=100,
                                        early_exit=isdc, vcycles=mode["vcycles"]))
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert rel_l2(host(u), ref) < 1e-12


def test_periodic_unsupported_combinations():
    from paper_1401_7824_amd import (Plan, Batch, ISDCError, STENCIL_COMPACT4 as SC, BC_PERIODIC as BP,
                                     KERNEL_EXPLICIT, KERNEL_TAIL, OP_EXPLICIT)
    announce("periodic unsupported")
    with pytest.raises(ISDCError):
        Plan(2, 32, 1.0, bc=BP)  # periodic second-order stencil
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, stencil=SC, bc=BP, smoother=1)  # not a power of two
    with pytest.raises(ISDCError):
        Plan(2, 2, 1.0, stencil=SC, bc=BP, smoother=1)  # below 4 points
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, FE_BURGERS, stencil=SC, smoother=1)  # Burgers on a Dirichlet grid
    p = Plan(2, 32, 1.0, stencil=SC, bc=BP, smoother=1)
    with pytest.raises(ISDCError):
        p.time_kernel(KERNEL_EXPLICIT, 0, 0.0, 0, 1)  # no stencil f^E in this plan
    with pytest.raises(ISDCError):
        p.mg_op(OP_EXPLICIT, 0, 0.0, a=dev(np.zeros((32, 32))), out=dev(np.zeros((32, 32))))
    us, nbytes = p.time_kernel(KERNEL_TAIL, 0, 1e-3, 0, 2)
    assert us > 0 and nbytes == 2 * 32 * 32 * 8
    q = Plan(2, 64, 1.0, FE_BURGERS, stencil=SC, bc=BP, smoother=1)
    us, nbytes = q.time_kernel(KERNEL_EXPLICIT, 0, 0.0, 0, 2)
    assert us > 0 and nbytes == 2 * 64 * 64 * 8
    b = Batch(2, 2)
    u = dev(np.zeros((32, 32)))
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, stencil=SC, bc=BP, smoother=1)
