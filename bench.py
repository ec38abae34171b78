#!/usr/bin/env python3
"""ISDC throughput on one MI355X: steps/s of the 2D reaction-diffusion workload.

Workload (default): u_t = nu Lap(u) + u - u^3 on [0,1]^2, Dirichlet, 1023^2
interior points, nu = 0.1, 16 seeded sine modes, Gauss-Lobatto M = 5,
dt = 1e-3, FP64, L = 2 RB-GS V(1,1) cycles per implicit solve, sweeps until
the SDC residual < 1e-10.  One "step" is one complete ISDC time step (all
sweeps, all V-cycles, the quadrature and the residual), with the state
resident in HBM; the timed steps continue the time integration.

Prints one JSON line.  Only one GPU is supported (--gpus 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ISDC steps/s, V-cycle HBM GB/s (% of peak), p50/p99 request latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rd2d", choices=["rd2d", "heat3d", "heat1d"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-reps", type=int, default=50)
    return ap.parse_args()


def make_plan(cfg):
    from paper_1401_7824_amd import Plan
    return Plan(cfg["dim"], cfg["n"], cfg["nu"], cfg["fe_kind"], node_kind=cfg["node_kind"], M=cfg["M"],
                precision=cfg["precision"], sdc_tol=cfg["sdc_tol"])


def time_steps(plan, u, dt, steps, warmup, torch):
    stream = torch.cuda.current_stream()
    stats = []
    for _ in range(warmup):
        plan.step(u, dt)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(steps):
        st = plan.step(u, dt)
        if st.status != "ok":
            raise RuntimeError(f"step failed: {st.status} after {st.sweeps} sweeps, residual {st.residual}")
        stats.append(st)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    return t0.elapsed_time(t1) / 1e3, wall, stats


def smoother_probe(plan, cfg, reps, torch):
    """Average duration of the fine-level one-pass red-black smoother
    (k_rbgs_tile), timed with HIP events on the stream it is launched on."""
    import paper_1401_7824_amd as P
    n, d = cfg["n"], cfg["dim"]
    dtype = torch.float64 if cfg["precision"] == 0 else torch.float32
    w = 8 if dtype == torch.float64 else 4
    g = torch.Generator(device="cuda").manual_seed(0)
    rhs = torch.randn((n,) * d, dtype=dtype, device="cuda", generator=g)
    u = [torch.randn((n,) * d, dtype=dtype, device="cuda", generator=g) for _ in range(2)]
    c = cfg["dt"] * cfg["nu"] * 0.3
    for k in range(4):
        plan.mg_op(P.OP_SMOOTH, 0, c, a=rhs, b=u[k % 2], out=u[(k + 1) % 2])
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(reps):
        plan.mg_op(P.OP_SMOOTH, 0, c, a=rhs, b=u[k % 2], out=u[(k + 1) % 2])
    e1.record(stream)
    torch.cuda.synchronize()
    per_launch = e0.elapsed_time(e1) / 1e3 / reps
    N = n ** d
    alg_bytes = 3 * w * N  # read the iterate and the right-hand side, write the new iterate
    achieved = alg_bytes / per_launch / 1e9
    return dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                kernel=f"k_rbgs_tile<{'double' if w == 8 else 'float'},{d},false> (fine level, {n}^{d})",
                avg_launch_us=round(per_launch * 1e6, 3), alg_bytes_per_launch=alg_bytes)


def cpu_baseline(cfg, sweeps_per_step):
    """The oracle (numpy, one thread) on a bounded sample: a few sweeps of one
    step at full size, scaled to steps/s with the GPU's sweeps per step."""
    import numpy as np
    import oracle as O  # noqa: F401  (test infrastructure: the CPU baseline only)
    from oracle.sdc import SDCConfig, sdc_begin, sdc_sweep
    from paper_1401_7824_amd import workloads as W
    u0 = W.workload_u0(cfg)
    sc = SDCConfig(nu=cfg["nu"], fe_kind=cfg["fe_kind"], node_kind=cfg["node_kind"], M=cfg["M"],
                   precision=cfg["precision"], tol=cfg["sdc_tol"])
    h = 1.0 / (cfg["n"] + 1)
    t0 = time.perf_counter()
    st = sdc_begin(u0, cfg["dt"], h, sc)
    nsw = 0
    while True:
        sdc_sweep(st)
        nsw += 1
        el = time.perf_counter() - t0
        if el > 10.0 or nsw >= sweeps_per_step:
            break
    per_sweep = el / nsw
    del np
    return dict(value=round(1.0 / (per_sweep * sweeps_per_step), 5), unit="steps/s", cores=1, kind="oracle",
                sample=f"{nsw} sweeps of one {cfg['n']}^{cfg['dim']} step on 1 host core "
                       f"({per_sweep:.2f} s/sweep), scaled by {sweeps_per_step:.1f} sweeps/step")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1401_7824_amd as P
    from paper_1401_7824_amd import workloads as W
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    P.load()
    cfg = dict(W.WORKLOADS[args.workload])
    plan = make_plan(cfg)
    u = torch.from_numpy(W.workload_u0(cfg)).cuda()
    elapsed, wall, stats = time_steps(plan, u, cfg["dt"], args.steps, args.warmup, torch)
    sweeps = sum(s.sweeps for s in stats) / len(stats)
    vcyc = sum(s.vcycles for s in stats) / len(stats)
    roof = smoother_probe(plan, cfg, args.probe_reps, torch)
    out = {
        "metric": METRIC,
        "value": round(args.steps / elapsed, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if cfg["precision"] == 0 else "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['dim']}D n={cfg['n']} nu={cfg['nu']} "
                               f"fe={'cubic' if cfg['fe_kind'] else 'zero'} "
                               f"{'Lobatto' if cfg['node_kind'] == 0 else 'Radau-right'} M={cfg['M']} "
                               f"dt={cfg['dt']} L=2 RBGS V(1,1) tol={cfg['sdc_tol']}",
                   "sweeps_per_step": sweeps, "vcycles_per_step": vcyc,
                   "host_wall_s": round(wall, 4)},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
