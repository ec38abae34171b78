"""GPU parity of two-level MLSDC with ISDC sweeps (Sec. 5) against the oracle.

Each iteration is a fine sweep, one coarse sweep on the (n-1)/2 grid with the
FAS term, and the coarse correction interpolated back (cubic).  The GPU forms
the coarse sweep's node-to-node sum as the injected fine S F, which equals
the oracle's S F_2h(R U) + tau_{m+1} - tau_m up to rounding.  FP64 iterates
agree to 1e-12 relative L2 and the iteration and V-cycle counts are equal.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle.mlsdc import mlsdc_step, mlsdc_iteration, MLSDCStats
from oracle.sdc import SDCConfig, sdc_begin
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

LOB, RAD, LEG = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT, O.NODES_LEGENDRE


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _plan(d, n, nu, fe, **kw):
    from paper_1401_7824_amd import Plan
    return Plan(d, n, nu, fe, levels=2, **kw)


def _cfg(nu, fe, **kw):
    keys = dict(node_kind="node_kind", M="M", vcycles="vcycles", inner_tol="inner_tol", early_exit="early_exit",
                sdc_tol="tol", max_sweeps="max_sweeps", smoother="smoother", nu_pre="nu1", nu_post="nu2",
                precision="precision")
    return SDCConfig(nu=nu, fe_kind=fe, inner="mg", **{keys[k]: v for k, v in kw.items()})


CASES = [
    # (name, d, n, nu, fe, dt, params)
    ("heat1d-lob3", 1, 127, 1.0, O.FE_ZERO, 0.01, dict(node_kind=LOB, M=3)),
    ("rd2d-lob5", 2, 127, 0.1, O.FE_CUBIC, 1e-3, dict(node_kind=LOB, M=5)),
    ("heat2d-255-rad3", 2, 255, 1.0, O.FE_ZERO, 1e-3, dict(node_kind=RAD, M=3)),
    ("heat3d-rad3", 3, 31, 1.0, O.FE_ZERO, 1e-3, dict(node_kind=RAD, M=3)),
    ("rd2d-leg3", 2, 63, 0.5, O.FE_CUBIC, 2e-3, dict(node_kind=LEG, M=3)),
    ("heat2d-n7-tail", 2, 7, 1.0, O.FE_ZERO, 1e-2, dict(node_kind=LOB, M=3)),
    ("heat2d-n3", 2, 3, 1.0, O.FE_ZERO, 1e-2, dict(node_kind=RAD, M=2)),
    ("rd2d-jacobi", 2, 127, 0.5, O.FE_CUBIC, 2e-3, dict(node_kind=LOB, M=3, smoother=1, nu_pre=2, nu_post=2)),
    # the Table 1 tolerances: an inner tolerance of 1e-9 leaves the SDC residual near 5e-10
    ("heat2d-classical", 2, 63, 10.0, O.FE_ZERO, 1e-3, dict(node_kind=LOB, M=3, vcycles=0, inner_tol=1e-9,
                                                           sdc_tol=5e-8)),
    ("heat2d-early", 2, 63, 10.0, O.FE_ZERO, 1e-3, dict(node_kind=LOB, M=3, early_exit=1, inner_tol=1e-9,
                                                       sdc_tol=5e-8)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_mlsdc_step_equals_oracle(case):
    name, d, n, nu, fe, dt, par = case
    announce("mlsdc step", name)
    par = dict(par)
    tol = par.pop("sdc_tol", 1e-10)
    h = 1.0 / (n + 1)
    u0 = 2.0 * W.sine_field(n, d, W.draw_modes(d, min(8, n ** d), seed=300 + d))
    p = _plan(d, n, nu, fe, sdc_tol=tol, **par)
    u = dev(u0)
    st = p.step(u, dt)
    ref, rst, _ = mlsdc_step(u0, dt, h, _cfg(nu, fe, sdc_tol=tol, **par))
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles, st.coarse_vcycles) == (rst.iterations, rst.vcycles, rst.coarse_vcycles)
    assert rel_l2(host(u), ref) < 1e-12


def test_mlsdc_iterates_equal_oracle():
    announce("mlsdc iterates")
    d, n, nu, dt, M = 2, 127, 1.0, 2e-3, 5
    h = 1.0 / (n + 1)
    u0 = W.sine_field(n, d, W.draw_modes(d, 8, seed=310))
    p = _plan(d, n, nu, O.FE_ZERO, node_kind=LOB, M=M)
    u = dev(u0)
    p.begin(u, dt)
    fine = sdc_begin(u0, dt, h, _cfg(nu, O.FE_ZERO, node_kind=LOB, M=M))
    stats = MLSDCStats()
    for k in range(4):
        rg = p.sweep()
        ro = mlsdc_iteration(fine, stats)
        assert abs(rg - ro) <= 1e-9 * ro + 1e-15, (k, rg, ro)
        for j in range(1, M + 1):
            assert rel_l2(host(p.node_values(j)), fine.U[j]) < 1e-12, (k, j)
    p.end(u)


def test_mlsdc_mixed_precision_reaches_collocation():
    announce("mlsdc mixed")
    d, n, nu, dt, M = 2, 255, 1.0, 2e-3, 3
    h = 1.0 / (n + 1)
    u0 = W.sine_field(n, d, W.draw_modes(d, 8, seed=311))
    coll = O.collocation_heat_modal(u0, dt, nu, h, LOB, M)
    p = _plan(d, n, nu, O.FE_ZERO, node_kind=LOB, M=M, precision=1, sdc_tol=1e-11)
    u = dev(u0)
    st = p.step(u, dt)
    assert st.status == "ok" and st.coarse_vcycles > 0
    assert rel_l2(host(u), coll) < 1e-8


def test_mlsdc_unsupported_and_invalid():
    from paper_1401_7824_amd import Plan, Batch, ISDCError, STENCIL_COMPACT4 as SC
    announce("mlsdc unsupported")
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, levels=3)
    with pytest.raises(ISDCError):
        Plan(2, 1, 1.0, levels=2)
    with pytest.raises(ISDCError):
        Plan(2, 31, 1.0, stencil=SC, smoother=1, levels=2)
    b = Batch(2, 2)
    u = dev(np.zeros((31, 31)))
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, levels=2)
