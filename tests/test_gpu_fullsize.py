"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times: the 2D reaction-diffusion workload (1023^2, Gauss-Lobatto
M = 5, FP64, weighted-Jacobi V(3,3) cycles) against the oracle sweep by sweep
and over its whole first step, and the 3D heat workload (255^3, right
Gauss-Radau M = 3, all-FP64 and float32 V-cycles) against the direct
collocation solution, which is known in closed form per sine mode."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle.sdc import SDCConfig, sdc_begin, sdc_sweep
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _plan_for(cfg, **over):
    from paper_1401_7824_amd import Plan
    kw = dict(node_kind=cfg["node_kind"], M=cfg["M"], precision=cfg["precision"], sdc_tol=cfg["sdc_tol"],
              smoother=cfg.get("smoother", 0), nu_pre=cfg.get("nu_pre", 1), nu_post=cfg.get("nu_post", 1))
    kw.update(over)
    return Plan(cfg["dim"], cfg["n"], cfg["nu"], cfg["fe_kind"], **kw)


def test_rd2d_full_size_sweeps_match_oracle():
    cfg = W.WORKLOADS["rd2d"]
    announce("fullsize rd2d", cfg["n"])
    u0 = W.workload_u0(cfg)
    p = _plan_for(cfg)
    st = sdc_begin(u0, cfg["dt"], 1.0 / (cfg["n"] + 1),
                   SDCConfig(nu=cfg["nu"], fe_kind=cfg["fe_kind"], node_kind=cfg["node_kind"], M=cfg["M"],
                             smoother=cfg.get("smoother", 0), nu1=cfg.get("nu_pre", 1), nu2=cfg.get("nu_post", 1)))
    u0d = dev(u0)
    p.begin(u0d, cfg["dt"])
    for k in range(2):
        rg = p.sweep()
        rc = sdc_sweep(st)
        assert abs(rg - rc) <= 1e-6 * rc
    for j in (2, cfg["M"]):
        assert rel_l2(host(p.node_values(j)), st.U[j]) < 1e-12
    p.end(torch.empty_like(u0d))
    # the whole step: the oracle continues its sweeps to the tolerance, and
    # the GPU step from u_0 gives the same counts and the same result
    res_hist = [rc]
    while rc >= cfg["sdc_tol"] and st.stats.sweeps < 100:
        rc = sdc_sweep(st)
        res_hist.append(rc)
    assert rc < cfg["sdc_tol"]
    u = dev(u0)
    s = p.step(u, cfg["dt"])
    assert s.status == "ok" and s.residual < cfg["sdc_tol"]
    if all(abs(r / cfg["sdc_tol"] - 1.0) > 1e-6 for r in res_hist):
        assert s.sweeps == st.stats.sweeps and s.vcycles == st.stats.vcycles
    assert s.vcycles == s.sweeps * (cfg["M"] - 1) * 2
    assert rel_l2(host(u), st.U[cfg["M"]]) < 1e-12


def test_heat3d_full_size_mixed_matches_collocation():
    cfg = W.WORKLOADS["heat3d"]
    n, d = cfg["n"], cfg["dim"]
    announce("fullsize heat3d", n)
    modes = W.workload_modes(cfg)
    u0 = W.sine_field(n, d, modes)
    p = _plan_for(cfg, precision=1)
    u = dev(u0)
    s = p.step(u, cfg["dt"])
    assert s.status == "ok"
    # direct collocation: every sine mode is multiplied by R(dt nu lambda_a)
    h = 1.0 / (n + 1)
    lam = [sum(-(4.0 / h ** 2) * np.sin(ai * np.pi * h / 2) ** 2 for ai in a) for _, a in modes]
    R = O.stability_function(cfg["dt"] * cfg["nu"] * np.array(lam), cfg["node_kind"], cfg["M"])
    coll = W.sine_field(n, d, [(amp * r, a) for (amp, a), r in zip(modes, R)])
    got = host(u)
    assert rel_l2(got, coll) < 1e-8
    # the same for the all-FP64 path
    p64 = _plan_for(cfg, precision=0)
    u64 = dev(u0)
    s64 = p64.step(u64, cfg["dt"])
    assert s64.status == "ok"
    assert rel_l2(host(u64), coll) < 1e-8
