#!/usr/bin/env python3
"""ISDC throughput on one MI355X.

Default workload (heat3d): u_t = Lap(u) on [0,1]^3, Dirichlet, 255^3
interior points (a working set of about 2 GB, far above the 256 MB Infinity
Cache), 32 seeded sine modes, right Gauss-Radau M = 3, dt = 1e-3, L = 2
red-black V(1,1) cycles per implicit solve, sweeps until the SDC residual
< 1e-10.  `value` is the all-float64 steps/s; the float32-V-cycle variant
runs beside it.  One "step" is one complete ISDC time step (all sweeps, all
V-cycles, the quadrature and the residual), with the state resident in HBM;
the timed steps continue the time integration.  The dominant kernel's
duration is taken inside the timed steps (each of its launches records its
own dispatch start and end into HIP events).

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
    ap.add_argument("--workload", default="heat3d", choices=["rd2d", "rd2d_compact", "rd2d_mlsdc", "heat3d", "heat1d", "burgers2d", "batch", "serve", "table1",
                             "table1b", "kernels", "compare"])
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-solo", type=int, default=2, help="solo lanes of the server (requests on their own plan)")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,0.9,1.1",
                    help="arrival rates swept, as fractions of the saturated capacity")
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="saturated capacity (req/s) from an earlier run: skips the saturated run and the sequential baselines")
    ap.add_argument("--serve-seq-sat", action="store_true",
                    help="with --serve-capacity: also run the one-at-a-time baseline with every request at t = 0")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-cycles", default="jacobi33", choices=["rbgs11", "jacobi33"],
                    help="V-cycles of the batched instances: red-black V(1,1) or weighted-Jacobi V(3,3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve-latency", action="store_true",
                    help="skip the short serving run that gives the headline line its p50/p99 latency")
    ap.add_argument("--probe-reps", type=int, default=100)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (reference kernel for HBM byte counters)")
    return ap.parse_args()


def mg_params(cfg):
    """Stencil, boundary and multigrid settings of a workload (defaults:
    second-order stencil, Dirichlet, red-black V(1,1))."""
    return dict(stencil=cfg.get("stencil", 0), bc=cfg.get("bc", 0), smoother=cfg.get("smoother", 0),
                nu_pre=cfg.get("nu_pre", 1), nu_post=cfg.get("nu_post", 1))


def grid_h(cfg, n=None):
    """Grid spacing: periodic [-1, 1) with n points, else (0, 1) with n interior points."""
    n = cfg["n"] if n is None else n
    return 2.0 / n if cfg.get("bc", 0) == 1 else 1.0 / (n + 1)


def tail_n(cfg):
    """Largest level the single-workgroup tail takes."""
    if cfg.get("bc", 0) == 1:
        return 32
    return {1: 2047, 2: 63, 3: 15}[cfg["dim"]]


def coarser(cfg, m):
    return m // 2 if cfg.get("bc", 0) == 1 else (m - 1) // 2


def make_plan(cfg):
    from paper_1401_7824_amd import Plan
    return Plan(cfg["dim"], cfg["n"], cfg["nu"], cfg["fe_kind"], node_kind=cfg["node_kind"], M=cfg["M"],
                precision=cfg["precision"], sdc_tol=cfg["sdc_tol"], levels=cfg.get("levels", 1), **mg_params(cfg))


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


KERNEL_NAMES = {
    "smooth_restrict": "k_rbgs_restrict_tile<{T},{d},false,{S}>",
    "prolong_smooth": "k_prolong_rbgs_tile<{T},{d},0,{S}>",
    "tail": "k_tail<{T},{d}>",
    "quad": "k_quad_residual_tile<{d},{M}>",
}


# 2D levels run the row-mapped tile kernels
ROW_KERNEL_NAMES = {
    "smooth": "k_rows_rbgs<{T},false,{S}>",
    "smooth_restrict": "k_rows_rbgs_restrict<{T},false,{S}>",
    "prolong_smooth": "k_rows_prolong_rbgs<{T},0,{S}>",
}


def kernel_name(name, cfg, T, shape=0):
    """rocprof name of the kernel bench.py times for `name` on the finest level
    (tile shape `shape`; 3D levels of 127^3 and up run the z-marching form)."""
    if cfg.get("stencil", 0) == 1:
        per = "true" if cfg.get("bc", 0) == 1 else "false"
        ks = min(3, max(1, cfg.get("nu_pre", 3)))
        return {"smooth": f"k_cjres<{T},{per},{ks},false>", "tail": f"k_ctail<{T},{per}>",
                "explicit": "k_weno_burgers"}[name]
    if cfg["dim"] == 3 and cfg["n"] >= 127 and name == "prolong_smooth":
        return f"k_march_rbgs<{T},true,0,false>"
    if cfg["dim"] == 2 and name in ROW_KERNEL_NAMES:
        return ROW_KERNEL_NAMES[name].format(T=T, S=shape)
    return KERNEL_NAMES[name].format(T=T, d=cfg["dim"], M=cfg["M"], S=shape)


def pade_exp(k, j):
    """Ascending coefficients of the (k, j) Pade approximant P/Q of exp(z)."""
    from math import factorial as f
    num = [f(k + j - i) * f(k) / (f(k + j) * f(i) * f(k - i)) for i in range(k + 1)]
    den = [(-1) ** i * f(k + j - i) * f(j) / (f(k + j) * f(i) * f(j - i)) for i in range(j + 1)]
    return num, den


def collocation_stability(node_kind, M, z):
    """R(z) of collocation with M nodes (Sec. 1) for u' = lambda u, z = dt lambda:
    Gauss-Lobatto collocation (Lobatto IIIA) gives the (M-1, M-1) Pade
    approximant of exp, right Gauss-Radau (Radau IIA) the (M-1, M) one,
    Gauss-Legendre the (M, M) one.  A textbook closed form, independent of the
    library's quadrature tables."""
    import numpy as np
    k, j = {0: (M - 1, M - 1), 1: (M - 1, M), 2: (M, M)}[node_kind]
    num, den = pade_exp(k, j)
    z = np.asarray(z, dtype=np.float64)
    return np.polyval(num[::-1], z) / np.polyval(den[::-1], z)


def collocation_reference(cfg, u0_modes, nsteps, n=None):
    """Direct collocation solution of a heat workload after nsteps steps: each
    sine mode of u_0 (an eigenvector of L_h with eigenvalue
    -(4/h^2) sum_i sin^2(a_i pi h / 2)) multiplied by R(dt nu lambda)^nsteps."""
    import numpy as np
    from paper_1401_7824_amd import workloads as W
    n = cfg["n"] if n is None else n
    d = cfg["dim"]
    h = 1.0 / (n + 1)
    lam = np.array([sum(-(4.0 / h ** 2) * np.sin(ai * np.pi * h / 2) ** 2 for ai in a) for _, a in u0_modes])
    R = collocation_stability(cfg["node_kind"], cfg["M"], cfg["dt"] * cfg["nu"] * lam)
    return W.sine_field(n, d, [(amp * r ** nsteps, a) for (amp, a), r in zip(u0_modes, R)])


def accuracy_vs_collocation(cfg, torch):
    """One step of a linear (heat) workload in float32-V-cycle and all-float64
    form, each compared with the direct collocation solution: the sine-mode
    expansion of u_0 with every mode multiplied by the collocation stability
    function R(z), z = dt nu lambda_a (Sec. 2), from its Pade closed form
    (collocation_stability).  Also times both variants."""
    import numpy as np
    from paper_1401_7824_amd import workloads as W
    n, d = cfg["n"], cfg["dim"]
    modes = W.workload_modes(cfg)
    u0 = W.sine_field(n, d, modes)
    coll = collocation_reference(cfg, modes, 1)
    out = {}
    for prec in (1, 0):
        c = dict(cfg, precision=prec)
        p = make_plan(c)
        u = torch.from_numpy(u0).cuda()
        st = p.step(u, cfg["dt"])
        got = u.cpu().numpy()
        err = float(np.linalg.norm(got - coll) / np.linalg.norm(coll))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            p.step(u, cfg["dt"])
        torch.cuda.synchronize()
        out["mixed" if prec else "fp64"] = dict(rel_l2_vs_collocation=err, sweeps=st.sweeps, status=st.status,
                                                 steps_per_s=round(3 / (time.perf_counter() - t0), 3))
    return out


# kernels followed inside the steps (isdc_probe_arm): (key, ISDC_KERNEL_*, level)
PROBE_KINDS = [("smooth", 2, 0), ("smooth_restrict", 0, 0), ("restrict", 7, 0), ("prolong_smooth", 1, 0),
               ("prolong_update", 6, 0), ("zsmooth_restrict", 9, 0), ("quad", 4, 0), ("rhs", 8, 0), ("tail", 3, 0)]


def probe_kernel_name(key, cfg, T, shape=0):
    """rocprof name of the finest-level kernel a probe key follows."""
    d, M = cfg["dim"], cfg["M"]
    if key == "quad":
        return f"k_quad_residual_tile<{d},{M}>"
    if key == "tail":
        return f"k_tail<{T},{d}>"
    if key == "rhs":
        return f"k_euler_rhs<{T},{d},0>"
    if d == 3 and cfg["n"] >= 127:
        return {"smooth": f"k_march_rbgs<{T},false,0,false>", "restrict": f"k_march_restrict<{T}>",
                "zsmooth_restrict": f"k_march_zrestrict<{T}>", "smooth_restrict": f"k_march_srestrict<{T}>",
                "prolong_smooth": f"k_march_rbgs<{T},true,0,false>",
                "prolong_update": f"k_march_rbgs<{T},true,1,false>"}[key]
    if d == 2 and cfg.get("smoother", 0) == 1:  # fused weighted-Jacobi row kernels of the five-point operator
        kpre, kpost = min(3, cfg.get("nu_pre", 2)), min(3, cfg.get("nu_post", 2))
        return {"smooth_restrict": f"k_cjres<{T},false,{kpre},false,false>",
                "prolong_smooth": f"k_cpjac<{T},false,{kpost},false,0>",
                "prolong_update": f"k_cpjac<{T},false,{kpost},false,1>"}[key]
    if d == 2:
        return {"smooth": f"k_rows_rbgs<{T},false,{shape}>", "smooth_restrict": f"k_rows_rbgs_restrict<{T},false,{shape}>",
                "zsmooth_restrict": f"k_rows_rbgs_restrict<{T},true,{shape}>",
                "prolong_smooth": f"k_rows_prolong_rbgs<{T},0,{shape}>",
                "prolong_update": f"k_rows_prolong_rbgs<{T},1,{shape}>"}[key]
    return {"smooth": f"k_rbgs_tile<{T},{d},false,{shape}>", "smooth_restrict": f"k_rbgs_restrict_tile<{T},{d},false,{shape}>",
            "zsmooth_restrict": f"k_rbgs_restrict_tile<{T},{d},true,{shape}>",
            "restrict": f"k_restrict_tile<{T},{d}>", "prolong_smooth": f"k_prolong_rbgs_tile<{T},{d},0,{shape}>",
            "prolong_update": f"k_prolong_rbgs_tile<{T},{d},1,{shape}>"}[key]


def kernel_survey(plan, u, dt, cfg):
    """Kernel time per step of each followed kernel: one step per kernel with
    every launch of that kernel recording its dispatch start and end (untimed
    steps before the warm-up; they continue the integration).  Returns
    ({key: (launches, average us, us per step, algorithmic bytes per launch)}, steps run)."""
    out = {}
    ran = 0
    for key, kind, level in PROBE_KINDS:
        try:
            plan.probe_arm(kind, level, 1, 100000)
        except Exception:
            continue  # not followed in this plan (e.g. no level above the tail)
        st = plan.step(u, dt)
        ran += 1
        if st.status != "ok":
            raise RuntimeError(f"survey step failed: {st.status}")
        n, us, b = plan.probe_read()
        if n:
            out[key] = (n, us, n * us, b)
    return out, ran


def counter_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on the finest level of `workload` from the
    committed FETCH_SIZE / WRITE_SIZE counter runs (profiles/traffic.json, written
    by paper_1401_7824_amd.profiling), or None if there is no such record or the
    kernel sources have changed since the counters were taken."""
    from paper_1401_7824_amd.profiling import sources_sha256
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(f"{workload}:{kernel}")
    if rec is None or rec.get("sources_sha256") != sources_sha256(ROOT):
        return None
    return rec["bytes_per_launch"]


def kernel_probe(plan, cfg, reps, torch):
    """Per-launch durations of the step's kernels, timed by the library with a
    pair of HIP events around every launch on the stream it launches on, with
    the workload's coefficient c = dt_m nu of the first non-degenerate substep."""
    import paper_1401_7824_amd as P
    from paper_1401_7824_amd.isdc import tables
    tau, _, _ = tables(cfg["node_kind"], cfg["M"])
    taus = [0.0] + list(tau)
    dtm = next(cfg["dt"] * (taus[m + 1] - taus[m]) for m in range(cfg["M"]) if taus[m + 1] > taus[m])
    c = dtm * cfg["nu"]
    prec = cfg["precision"]
    T = "double" if prec == 0 else "float"
    out = {}
    kinds = [("smooth_restrict", P.KERNEL_SMOOTH_RESTRICT), ("prolong_smooth", P.KERNEL_PROLONG_SMOOTH),
             ("tail", P.KERNEL_TAIL)]
    if cfg.get("stencil", 0) == 1:  # compact plans: the weighted-Jacobi step and the compact tail
        kinds = [("smooth", P.KERNEL_SMOOTH), ("tail", P.KERNEL_TAIL)]
    if cfg["fe_kind"] == 2:  # the WENO5 Burgers advection
        kinds.append(("explicit", P.KERNEL_EXPLICIT))
    for name, k in kinds:
        if name == "smooth_restrict" and cfg["dim"] == 3:
            continue
        if name not in ("tail", "explicit") and cfg["n"] <= tail_n(cfg):
            continue  # the whole V-cycle is the single-workgroup coarse solve
        us, b = plan.time_kernel(k, 0, c, prec, reps)
        shape = (plan.tile_shapes or [0])[0]
        out[name] = dict(kernel=kernel_name(name, cfg, T, shape), avg_us=round(us, 3),
                         alg_bytes=b, gbps=round(b / (us * 1e-6) / 1e9, 1))
    return out


def vcycle_probe(plan, cfg, reps, torch):
    """Time of one whole fine-level V-cycle (isdc_vcycle, events on torch's
    stream) and its algorithmic HBM bytes: every level's arrays read or
    written once per kernel, summed over the levels the kernels touch."""
    n, d = cfg["n"], cfg["dim"]
    dtype = torch.float64 if cfg["precision"] == 0 else torch.float32
    w = 8 if dtype == torch.float64 else 4
    g = torch.Generator(device="cuda").manual_seed(0)
    rhs = torch.randn((n,) * d, dtype=dtype, device="cuda", generator=g)
    u = torch.zeros_like(rhs)
    c = cfg["dt"] * cfg["nu"] * 0.3
    for _ in range(3):
        plan.vcycle(c, rhs, u, 1)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        plan.vcycle(c, rhs, u, 1)
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    # per multi-workgroup level: (3N + Nc) for smoothing+restriction and for
    # prolongation+smoothing; the tail reads its rhs and writes its iterate
    b, m = 0.0, n
    compact = cfg.get("stencil", 0) == 1
    # compact: Jacobi steps + residual + restriction and prolongation + Jacobi
    # steps (3N + Nc each, up to three steps per launch), further launches of
    # up to three steps 3N each
    extra = (-(-cfg.get("nu_pre", 1) // 3) - 1) + (-(-cfg.get("nu_post", 1) // 3) - 1)
    while m > tail_n(cfg):
        N, Nc = m ** d, coarser(cfg, m) ** d
        if compact:
            b += (2 * (3 * N + Nc) + extra * 3 * N) * w
        else:        # smoothing + restriction 3N + Nc; prolongation + smoothing 3N + Nc
            b += 2 * (3 * N + Nc) * w
        m = coarser(cfg, m)
    b += 2 * m ** d * w
    return dict(us_per_vcycle=round(us, 2), alg_bytes=b, gbps=round(b / (us * 1e-6) / 1e9, 1),
                frac=round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4))


def cpu_baseline(cfg, sweeps_per_step):
    """The oracle (numpy, one thread) on a bounded sample: sweeps of one step
    at full size, scaled to steps/s with the GPU's sweeps per step.  Above
    2^22 points a single full-size sweep would exceed the sample budget, so
    the sample runs on the next coarser grid (side (n-1)/2, or n/2 periodic)
    and is scaled by the ratio of point counts (the oracle's work is linear in
    the points)."""
    import numpy as np
    import oracle as O  # noqa: F401  (test infrastructure: the CPU baseline only)
    from oracle.sdc import SDCConfig, sdc_begin, sdc_sweep
    from oracle.mlsdc import MLSDCStats, mlsdc_iteration
    from paper_1401_7824_amd import workloads as W
    c = dict(cfg)
    scale = 1.0
    while c["n"] ** c["dim"] > 2 ** 22:
        small = coarser(c, c["n"])
        scale *= (c["n"] / small) ** c["dim"]
        c["n"] = small
    u0 = W.workload_u0(c)
    sc = SDCConfig(nu=c["nu"], fe_kind=c["fe_kind"], node_kind=c["node_kind"], M=c["M"],
                   precision=c["precision"], tol=c["sdc_tol"], stencil=c.get("stencil", 0), bc=c.get("bc", 0),
                   smoother=c.get("smoother", 0), nu1=c.get("nu_pre", 1), nu2=c.get("nu_post", 1))
    h = grid_h(c)
    t0 = time.perf_counter()
    st = sdc_begin(u0, c["dt"], h, sc)
    ml = MLSDCStats() if c.get("levels", 1) == 2 else None
    nsw = 0
    while True:
        if ml is not None:
            mlsdc_iteration(st, ml)  # one two-level iteration counts as one sweep
        else:
            sdc_sweep(st)
        nsw += 1
        el = time.perf_counter() - t0
        if el > 10.0 or nsw >= sweeps_per_step:
            break
    per_sweep = el / nsw * scale
    del np
    where = f"one {c['n']}^{c['dim']} step" + (f", scaled x{scale:.2f} to {cfg['n']}^{cfg['dim']}" if scale != 1 else "")
    return dict(value=round(1.0 / (per_sweep * sweeps_per_step), 6), unit="steps/s", cores=1, kind="oracle",
                sample=f"{nsw} sweeps of {where} on 1 host core ({per_sweep:.2f} s/sweep), "
                       f"scaled by {sweeps_per_step:.1f} sweeps/step")


def _oracle_instance_steps(job):
    """One oracle step of one batched instance (a process-pool task of the batch CPU baseline)."""
    import numpy as np
    from oracle.sdc import SDCConfig, sdc_step
    from paper_1401_7824_amd import workloads as W
    x = job
    u0 = W.sine_field(x["n"], 2, W.draw_modes(2, x["n_modes"], x["seed"]))
    cfg = SDCConfig(nu=x["nu"], fe_kind=x["fe_kind"], node_kind=x["node_kind"], M=x["M"], precision=x["precision"],
                    tol=x["sdc_tol"], max_sweeps=200)
    t0 = time.perf_counter()
    _, st = sdc_step(u0, x["dt"], 1.0 / (x["n"] + 1), cfg)
    del np
    return time.perf_counter() - t0, st.sweeps


def batch_cpu_baseline(inst, budget_s=20.0):
    """The oracle on the host cores (a process pool, one instance step per task) over a
    bounded sample of the batched instances, in instance-steps/s: every fourth
    instance is sampled until the pool has spent about budget_s seconds of wall time."""
    import multiprocessing as mp
    cores = min(16, len(os.sched_getaffinity(0)))  # the GPU host's CPU share is 16 cores
    sample = inst[::4]
    t0 = time.perf_counter()
    done = 0
    with mp.get_context("spawn").Pool(cores) as pool:
        for _ in pool.imap_unordered(_oracle_instance_steps, sample):
            done += 1
            if time.perf_counter() - t0 > budget_s:
                pool.terminate()
                break
    el = time.perf_counter() - t0
    return dict(value=round(done / el, 4), unit="instance-steps/s", cores=cores, kind="oracle",
                sample=f"{done} one-step tasks of every fourth batched instance (sides 63..511) in a pool of "
                       f"{cores} processes, {el:.1f} s wall")


def run_batch(args, torch):
    """256 uneven 2D reaction-diffusion instances (side 63..511, nu, dt, M drawn
    per instance, float32 V-cycles, tolerance 1e-8), each advanced
    --batch-steps steps: all in one batch, then one instance after another with
    isdc_step.  Reports both throughputs in instance-steps/s and checks that
    the two give bitwise the same states."""
    import numpy as np
    from paper_1401_7824_amd import Batch, Plan
    from paper_1401_7824_amd import workloads as W
    inst = W.batch_instances(args.batch_count)
    u0s = [W.sine_field(x["n"], 2, W.draw_modes(2, x["n_modes"], x["seed"])) for x in inst]
    steps = args.batch_steps
    cyc = dict(smoother=1, nu_pre=3, nu_post=3) if args.batch_cycles == "jacobi33" else {}
    par = lambda x: dict(node_kind=x["node_kind"], M=x["M"], precision=x["precision"], sdc_tol=x["sdc_tol"],  # noqa: E731
                         **cyc)
    b = Batch(len(inst), 2, precision=1, vcycles=2)
    ws = [torch.empty(Batch.workspace_bytes_for(x["n"], 2, x["nu"], x["fe_kind"], **par(x)), dtype=torch.uint8,
                      device="cuda") for x in inst]
    # launch schedule of one batch sweep of all 256 slots: kernel by kernel, as
    # isdc_batch_advance runs it, against one HIP graph replayed (measurement only)
    side = torch.cuda.Stream()
    ub = [torch.from_numpy(u).cuda() for u in u0s]
    for i, x in enumerate(inst):
        b.set(i, ub[i], x["dt"], steps, x["nu"], x["fe_kind"], workspace=ws[i], **par(x))
    torch.cuda.synchronize()
    b.advance(side)
    eager_us, launches = b.time_sweeps(10, False, side)
    graph_us, _ = b.time_sweeps(10, True, side)
    for i in range(len(inst)):
        b.release(i)
    torch.cuda.synchronize()
    print(f"[batch] sweep of {len(inst)} slots: {launches} launches, eager {eager_us:.1f} us, "
          f"graph {graph_us:.1f} us", file=sys.stderr, flush=True)
    # warm-up of every kernel shape on a copy
    for rep in range(2):
        ub = [torch.from_numpy(u).cuda() for u in u0s]
        for i, x in enumerate(inst):
            b.set(i, ub[i], x["dt"], 1 if rep == 0 else steps, x["nu"], x["fe_kind"], workspace=ws[i], **par(x))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sweeps = b.run()
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
    states = [b.info(i) for i in range(len(inst))]
    assert all(st[1] == "ok" for st in states), [st[1] for st in states]
    # one instance after another
    uref = [torch.from_numpy(u).cuda() for u in u0s]
    plans = {}
    t0 = time.perf_counter()
    for i, x in enumerate(inst):
        key = (x["n"], x["M"])
        p = Plan(2, x["n"], x["nu"], x["fe_kind"], **par(x))
        for _ in range(steps):
            st = p.step(uref[i], x["dt"])
            assert st.status == "ok"
        plans[key] = p
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    same = all(torch.equal(ub[i], uref[i]) for i in range(len(inst)))
    total = len(inst) * steps
    out = {
        "metric": METRIC, "value": round(total / t_batch, 3), "unit": "instance-steps/s", "n_gpus": 1,
        "steps": total, "warmup": 1, "ms_per_step": round(t_batch / total * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"batch: {len(inst)} 2D reaction-diffusion instances, side 63..511, "
                               f"{steps} steps each, float32 "
                               f"{'weighted-Jacobi V(3,3)' if cyc else 'red-black V(1,1)'} V-cycles, tol 1e-8",
                   "batch_sweeps": sweeps, "sizes": {str(k): sum(1 for x in inst if x['n'] == k) for k in (63, 127, 255, 511)}},
        "per_instance_baseline": {"value": round(total / t_single, 3), "unit": "instance-steps/s",
                                  "seconds": round(t_single, 3)},
        "speedup_vs_per_instance": round(t_single / t_batch, 2),
        "bitwise_equal_to_per_instance": bool(same),
        "sweep_launch_schedule": {"launches_per_sweep": launches, "eager_us_per_sweep": round(eager_us, 1),
                                  "hip_graph_us_per_sweep": round(graph_us, 1),
                                  "kept": "eager: the captured graph is within 3 % and would need a new capture "
                                          "whenever slots join or leave" if graph_us > 0.97 * eager_us
                                  else "graph is more than 3 % faster here"},
        "batch_seconds": round(t_batch, 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = batch_cpu_baseline(inst)
    return out


def serve_accuracy(reqs, torch, rd_sample=8):
    """Error of each served result (float32 V-cycles, the request's own SDC
    tolerance) against a float64 reference, relative L2: every heat request
    against the exact collocation solution after nsteps steps (each sine mode
    of u_0 multiplied by R(dt nu lambda)^nsteps, R the Pade closed form of the
    collocation stability function; the reference field is built on the
    device); reaction-diffusion requests (the rd_sample smallest) against an
    all-float64 plan run to SDC tolerance 1e-12."""
    import numpy as np
    from paper_1401_7824_amd import Plan, workloads as W
    rows = []
    for r in reqs:
        if r.result is None or r.status != "ok" or r.fe_kind != 0:
            continue
        h = 1.0 / (r.n + 1)
        lam = np.array([sum(-(4.0 / h ** 2) * np.sin(ai * np.pi * h / 2) ** 2 for ai in a) for _, a in r.modes])
        R = collocation_stability(r.node_kind, r.M, r.dt * r.nu * lam)
        ref = W.sine_field_device(r.n, r.dim, [(r.scale * amp * Rk ** r.nsteps, a) for (amp, a), Rk in zip(r.modes, R)])
        err = (torch.linalg.vector_norm(r.result - ref) / torch.linalg.vector_norm(ref)).item()
        rows.append(dict(rid=r.rid, dim=r.dim, n=r.n, tol=r.sdc_tol, steps=r.nsteps, kind="heat vs exact collocation",
                         rel_l2=float(err)))
    rd = sorted((r for r in reqs if r.fe_kind == 1 and r.result is not None and r.status == "ok"),
                key=lambda r: r.n ** r.dim)[:rd_sample]
    for r in rd:
        p = Plan(r.dim, r.n, r.nu, r.fe_kind, node_kind=r.node_kind, M=r.M, sdc_tol=1e-12, max_sweeps=400,
                 precision=0)
        u = r.u0_device()
        for _ in range(r.nsteps):
            p.step(u, r.dt)
        err = (torch.linalg.vector_norm(r.result - u) / torch.linalg.vector_norm(u)).item()
        rows.append(dict(rid=r.rid, dim=r.dim, n=r.n, tol=r.sdc_tol, steps=r.nsteps,
                         kind="reaction-diffusion vs float64 at tol 1e-12", rel_l2=float(err)))
    worst = {}
    for row in rows:
        key = f"tol {row['tol']:g}, {row['kind']}"
        worst[key] = max(worst.get(key, 0.0), row["rel_l2"])
    return {"checked": len(rows), "max_rel_l2_by_tolerance": worst,
            "per_result": rows if len(rows) <= 200 else "omitted (more than 200 results)"}


def run_serve(args, torch):
    """Serving: Poisson arrivals of mixed 2D (127^2..1023^2) and 3D (31^3..255^3)
    heat / reaction-diffusion requests (tolerance 1e-5 or 1e-8, 1..20 steps),
    admitted under an HBM budget into continuously batched slots.  The
    saturated capacity is measured first (all requests at t = 0); then the
    arrival rate is swept at 0.25 .. 1.1 of it, reporting p50 / p99 latency;
    the one-request-at-a-time baseline runs at the lowest rate."""
    from paper_1401_7824_amd.serve import Server, make_requests, serve_sequential
    budget = int(args.serve_budget_gb * 2 ** 30)
    count = args.serve_count

    def server():
        return Server(budget, slots_per_batch=64, precision=1, vcycles=2, solo_workers=args.serve_solo)

    log = max(1, count // 10)
    warm = make_requests(8, rate=0.0, seed=99)
    server().serve(warm)
    given = args.serve_capacity > 0
    if given:
        cap, sat, accuracy = args.serve_capacity, None, None
    else:
        sat_reqs = make_requests(count, rate=0.0, seed=5)
        sat = server().serve(sat_reqs, log_every=log)
        cap = sat.completed / sat.makespan
        accuracy = serve_accuracy(sat_reqs, torch)
        del sat_reqs
        print(f"[serve] saturated: {sat.completed} requests in {sat.makespan:.2f} s", file=sys.stderr, flush=True)
    rows = []
    for frac in [float(x) for x in args.serve_rates.split(",") if x]:
        reqs = make_requests(count, rate=frac * cap, seed=5)
        st = server().serve(reqs, log_every=log).summary()
        st["rate_req_s"] = round(frac * cap, 3)
        st["rate_frac_of_capacity"] = frac
        rows.append(st)
        print(f"[serve] rate {frac:.2f} x capacity: p50 {st['p50_ms']} ms, p99 {st['p99_ms']} ms",
              file=sys.stderr, flush=True)
    if given:
        out = {"metric": METRIC, "value": round(cap, 4), "unit": "requests/s", "n_gpus": 1, "steps": 0,
               "warmup": 8, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64+f32", "data": "synthetic",
               "config": {"workload": f"serve rate sweep only: {count} requests, capacity {cap} req/s given, HBM "
                                      f"budget {args.serve_budget_gb} GiB, {args.serve_solo} solo lanes"},
               "rate_sweep": rows}
        if args.serve_seq_sat:
            from paper_1401_7824_amd.serve import runs_solo
            seq_reqs = make_requests(count, rate=0.0, seed=5)
            seq_sat = serve_sequential(seq_reqs, precision=1, vcycles=2, log_every=log).summary()
            seq_sat["service_s_large_requests"] = round(
                sum(r.finished - r.admitted for r in seq_reqs if runs_solo(r, 1)), 3)
            seq_sat["service_s_other_requests"] = round(
                sum(r.finished - r.admitted for r in seq_reqs if not runs_solo(r, 1)), 3)
            out["sequential_baseline_saturated"] = seq_sat
            out["capacity_vs_sequential"] = round(cap / seq_sat["throughput_req_s"], 2)
            print(f"[serve] sequential saturated: {seq_sat['throughput_req_s']} req/s", file=sys.stderr, flush=True)
        return out
    seq = serve_sequential(make_requests(count, rate=0.25 * cap, seed=5), precision=1, vcycles=2,
                           log_every=log).summary()
    print(f"[serve] sequential at 0.25 x capacity: p50 {seq['p50_ms']} ms, p99 {seq['p99_ms']} ms",
          file=sys.stderr, flush=True)
    seq_reqs = make_requests(count, rate=0.0, seed=5)
    seq_sat = serve_sequential(seq_reqs, precision=1, vcycles=2, log_every=log).summary()
    # where the one-at-a-time time goes: requests the server runs solo (large grids) against the rest
    from paper_1401_7824_amd.serve import runs_solo
    big = sum(r.finished - r.admitted for r in seq_reqs if runs_solo(r, 1))
    small = sum(r.finished - r.admitted for r in seq_reqs if not runs_solo(r, 1))
    seq_sat["service_s_large_requests"] = round(big, 3)
    seq_sat["service_s_other_requests"] = round(small, 3)
    print(f"[serve] sequential saturated: {seq_sat['throughput_req_s']} req/s", file=sys.stderr, flush=True)
    steps = sum(r.nsteps for r in make_requests(count, rate=0.0, seed=5))
    return {
        "metric": METRIC, "value": round(cap, 4), "unit": "requests/s", "n_gpus": 1, "steps": steps,
        "warmup": 8, "ms_per_step": round(sat.makespan / steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"serve: {count} requests, half 2D 127..1023, half 3D 31..255, heat / "
                               f"reaction-diffusion, tol 1e-5 / 1e-8, 1..20 steps, HBM budget "
                               f"{args.serve_budget_gb} GiB, 64 slots per dimension, {args.serve_solo} solo lanes"},
        "saturated": sat.summary(), "accuracy": accuracy, "rate_sweep": rows, "sequential_baseline_at_0.25": seq,
        "sequential_baseline_saturated": seq_sat,
        "capacity_vs_sequential": round(cap / seq_sat["throughput_req_s"], 2) if seq_sat["throughput_req_s"] else None,
    }


def run_kernels(args, torch):
    """Streaming efficiency of the fine-level multigrid kernels against grid
    size: per-launch time of each kernel (HIP events around every launch,
    isdc_time_kernel), its algorithmic bytes (each array it touches read or
    written once) and the achieved GB/s, beside a plain device-to-device copy
    of one array of the same size.  Working sets from inside the 256 MB
    Infinity Cache (1023^2) to far outside it (8191^2, 511^3)."""
    import paper_1401_7824_amd as P
    from paper_1401_7824_amd import Plan
    rows = []
    cases = [(2, n, prec) for n in (1023, 2047, 4095, 8191) for prec in (0, 1)] + \
            [(3, n, prec) for n in (255, 511) for prec in (0, 1)]
    for d, n, prec in cases:
        p = Plan(d, n, 1.0, 0, node_kind=0, M=3, precision=prec)
        c = 1e-3 * 0.5
        row = {"dim": d, "n": n, "dtype": "f64" if prec == 0 else "f32"}
        # the fused smoothing + restriction runs on 2D levels and on z-marched 3D levels
        kinds = [("smooth_restrict", P.KERNEL_SMOOTH_RESTRICT), ("smooth", P.KERNEL_SMOOTH),
                 ("prolong_smooth", P.KERNEL_PROLONG_SMOOTH)]
        nl = len(p.tile_shapes)
        shapes = range(3)  # tile shapes (3D levels of 127^3 and up: column depths of the z-march)
        for name, k in kinds:
            best = None
            for sh in shapes:  # every tile shape on the finest level; the fastest is reported
                p.tile_shapes = [sh] * nl
                us, b = p.time_kernel(k, 0, c, prec, args.probe_reps)
                if best is None or us < best[0]:
                    best = (us, b, sh)
            us, b, sh = best
            row[name] = {"us": round(us, 2), "alg_bytes": int(b), "gbps": round(b / (us * 1e-6) / 1e9, 1),
                         "frac": round(b / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "shape": sh}
        dt = torch.float64 if prec == 0 else torch.float32
        src = torch.empty((n,) * d, dtype=dt, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.probe_reps):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / args.probe_reps
        row["copy"] = {"us": round(us, 2), "gbps": round(2 * src.numel() * src.element_size() / (us * 1e-6) / 1e9, 1)}
        rows.append(row)
        print(f"[kernels] {d}D n={n} {row['dtype']}: " + ", ".join(
            f"{k} {v['gbps']} GB/s" + (f" (shape {v['shape']})" if "shape" in v else "")
            for k, v in row.items() if isinstance(v, dict)), file=sys.stderr, flush=True)
        del p, src, dst
        torch.cuda.empty_cache()
    big = [r for r in rows if r["dim"] == 2 and r["n"] == 8191 and r["dtype"] == "f64"][0]
    best = big["smooth_restrict"]
    return {
        "metric": METRIC, "value": best["gbps"], "unit": "GB/s", "n_gpus": 1, "steps": args.probe_reps,
        "warmup": 1, "ms_per_step": round(best["us"] / 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "kernels: fine-level multigrid kernels, 2D 1023^2..8191^2 and 3D 255^3..511^3, "
                               "f64 and f32; value = fused smoothing + restriction at 8191^2 f64"},
        "roofline": {"bound": "hbm", "achieved": best["gbps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": best["frac"], "traffic": None,
                     "kernel": f"k_rbgs_restrict_tile<double,2,false,{best['shape']}> (8191^2)",
                     "avg_launch_us": best["us"], "alg_bytes_per_launch": best["alg_bytes"]},
        "rows": rows,
    }


def run_table1(args, torch):
    """Table 1(a) replay (Sec. 4): 2D heat on [0,1]^2, u0 = sin(pi x) sin(pi y),
    n = 63 (h = 1/64), dt = 1e-3, Gauss-Lobatto M in {3, 5, 7}, nu in
    {1, 10, 100}, sweeps until the max-norm SDC residual < 5e-8, with the
    fourth-order compact stencil and weighting matrix W of the paper's runs
    (eq. (5)) and with the second-order stencil.  Multigrid: weighted-Jacobi
    V(3,3) (omega = 1 compact, 4/5 second order).  Classical SDC cycles each
    implicit solve until its max-norm residual <= 1e-9; ISDC stops after
    L = 2 cycles or earlier at that tolerance.  Reports accumulated V-cycles
    and sweeps beside the printed ones and the GPU time of one step of each;
    `value` is the compact stencil's V-cycle saving summed over the nine rows."""
    import csv
    import numpy as np
    from paper_1401_7824_amd import Plan
    n, dt = 63, 1e-3
    x = np.arange(1, n + 1) / (n + 1)
    u0 = np.outer(np.sin(np.pi * x), np.sin(np.pi * x))
    printed = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1.csv")) as fh:
        for r in csv.DictReader(line for line in fh if not line.startswith("#")):
            if r["problem"] == "heat":
                printed[(float(r["nu"]), int(r["M"]))] = r
    out = {}
    for sname, stencil in (("compact4", 1), ("second_order", 0)):
        rows = []
        tot = {"sdc": 0, "isdc": 0}
        ms_tot = {"sdc": 0.0, "isdc": 0.0}
        for nu in (1.0, 10.0, 100.0):
            for M in (3, 5, 7):
                row = {"nu": nu, "M": M}
                for name, mode in (("sdc", dict(vcycles=0)), ("isdc", dict(vcycles=2, early_exit=1))):
                    p = Plan(2, n, nu, 0, stencil=stencil, node_kind=0, M=M, sdc_tol=5e-8, inner_tol=1e-9,
                             max_sweeps=100, smoother=1, nu_pre=3, nu_post=3, **mode)
                    u0d = torch.from_numpy(u0).cuda()
                    u = u0d.clone()
                    st = p.step(u, dt)
                    reps = max(1, args.steps)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(reps):
                        u.copy_(u0d)
                        p.step(u, dt)
                    torch.cuda.synchronize()
                    ms = (time.perf_counter() - t0) / reps * 1e3
                    row[name] = {"vcycles": st.vcycles, "sweeps": st.sweeps, "status": st.status,
                                 "ms_per_step": round(ms, 3)}
                    tot[name] += st.vcycles
                    ms_tot[name] += ms
                pr = printed[(nu, M)]
                row["savings_pct"] = round(100.0 * (1 - row["isdc"]["vcycles"] / row["sdc"]["vcycles"]), 1)
                row["time_savings_pct"] = round(100.0 * (1 - row["isdc"]["ms_per_step"] / row["sdc"]["ms_per_step"]), 1)
                row["printed"] = {"sdc": f"{pr['sdc_cycles']}({pr['sdc_sweeps']})",
                                  "isdc": f"{pr['isdc_cycles']}({pr['isdc_sweeps']})",
                                  "savings_pct": int(pr["savings_pct"])}
                rows.append(row)
                print(f"[table1 {sname}] nu={nu:5.0f} M={M}: SDC {row['sdc']['vcycles']}({row['sdc']['sweeps']}) "
                      f"ISDC {row['isdc']['vcycles']}({row['isdc']['sweeps']}) save {row['savings_pct']}% | "
                      f"printed {row['printed']['sdc']} {row['printed']['isdc']} {pr['savings_pct']}%",
                      file=sys.stderr, flush=True)
        out[sname] = {"savings_pct": round(100.0 * (1 - tot["isdc"] / tot["sdc"]), 2),
                      "time_savings_pct": round(100.0 * (1 - ms_tot["isdc"] / ms_tot["sdc"]), 2),
                      "totals": {"sdc_vcycles": tot["sdc"], "isdc_vcycles": tot["isdc"],
                                 "sdc_ms": round(ms_tot["sdc"], 3), "isdc_ms": round(ms_tot["isdc"], 3)},
                      "rows": rows}
    printed_save = 100.0 * (1 - sum(int(r["isdc_cycles"]) for r in printed.values())
                            / sum(int(r["sdc_cycles"]) for r in printed.values()))
    c4 = out["compact4"]
    return {
        "metric": "Table 1(a) replay: accumulated V-cycles of classical SDC vs ISDC", "value": c4["savings_pct"],
        "unit": "% V-cycles saved (9 rows)", "n_gpus": 1, "steps": 36 * max(1, args.steps), "warmup": 36,
        "ms_per_step": round((c4["totals"]["sdc_ms"] + c4["totals"]["isdc_ms"]) / 18, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "table1: 2D heat n=63 (h=1/64) u0=sin(pi x)sin(pi y) dt=1e-3 Lobatto M=3,5,7 "
                               "nu=1,10,100 tol 5e-8; SDC inner_tol 1e-9; ISDC L=2 early exit; weighted-Jacobi "
                               "V(3,3); value: fourth-order compact stencil with W"},
        "printed_savings_pct_9_rows": round(printed_save, 2),
        "stencils": out,
    }


def run_table1b(args, torch):
    """Table 1(b) replay (Sec. 4.1): 2D viscous Burgers on [-1, 1)^2, periodic,
    n = 128 (h = 1/64, diffusive CFL 0.41 / 4.1 / 41), u0 = exp(-|x|^2 / 0.1^2),
    WENO5 advection, fourth-order compact stencil with W, dt = 1e-3,
    Gauss-Lobatto M in {3, 5, 7}, nu in {0.1, 1, 10}, sweeps until the max-norm
    SDC residual < 5e-8; weighted-Jacobi V(3,3) (omega = 1).  Classical SDC
    cycles each implicit solve until its max-norm residual <= 1e-9; ISDC stops
    after L = 2 cycles or earlier at that tolerance.  `value` is the V-cycle
    saving summed over the nine rows."""
    import csv
    from paper_1401_7824_amd import Plan, workloads as W
    n, dt = 128, 1e-3
    u0 = W.gaussian_periodic(n, 0.1)
    printed = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1.csv")) as fh:
        for r in csv.DictReader(line for line in fh if not line.startswith("#")):
            if r["problem"] == "burgers":
                printed[(float(r["nu"]), int(r["M"]))] = r
    rows = []
    tot = {"sdc": 0, "isdc": 0}
    ms_tot = {"sdc": 0.0, "isdc": 0.0}
    for nu in (0.1, 1.0, 10.0):
        for M in (3, 5, 7):
            row = {"nu": nu, "M": M}
            for name, mode in (("sdc", dict(vcycles=0)), ("isdc", dict(vcycles=2, early_exit=1))):
                p = Plan(2, n, nu, W.FE_BURGERS, stencil=1, bc=1, node_kind=0, M=M, sdc_tol=5e-8, inner_tol=1e-9,
                         max_sweeps=100, smoother=1, nu_pre=3, nu_post=3, **mode)
                u0d = torch.from_numpy(u0).cuda()
                u = u0d.clone()
                st = p.step(u, dt)
                reps = max(1, args.steps)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    u.copy_(u0d)
                    p.step(u, dt)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / reps * 1e3
                row[name] = {"vcycles": st.vcycles, "sweeps": st.sweeps, "status": st.status,
                             "ms_per_step": round(ms, 3)}
                tot[name] += st.vcycles
                ms_tot[name] += ms
            pr = printed[(nu, M)]
            row["savings_pct"] = round(100.0 * (1 - row["isdc"]["vcycles"] / row["sdc"]["vcycles"]), 1)
            row["time_savings_pct"] = round(100.0 * (1 - row["isdc"]["ms_per_step"] / row["sdc"]["ms_per_step"]), 1)
            row["printed"] = {"sdc": f"{pr['sdc_cycles']}({pr['sdc_sweeps']})",
                              "isdc": f"{pr['isdc_cycles']}({pr['isdc_sweeps']})",
                              "savings_pct": int(pr["savings_pct"])}
            rows.append(row)
            print(f"[table1b] nu={nu:5.1f} M={M}: SDC {row['sdc']['vcycles']}({row['sdc']['sweeps']}) "
                  f"ISDC {row['isdc']['vcycles']}({row['isdc']['sweeps']}) save {row['savings_pct']}% | "
                  f"printed {row['printed']['sdc']} {row['printed']['isdc']} {pr['savings_pct']}%",
                  file=sys.stderr, flush=True)
    printed_save = 100.0 * (1 - sum(int(r["isdc_cycles"]) for r in printed.values())
                            / sum(int(r["sdc_cycles"]) for r in printed.values()))
    return {
        "metric": "Table 1(b) replay: accumulated V-cycles of classical SDC vs ISDC",
        "value": round(100.0 * (1 - tot["isdc"] / tot["sdc"]), 2),
        "unit": "% V-cycles saved (9 rows)", "n_gpus": 1, "steps": 18 * max(1, args.steps), "warmup": 18,
        "ms_per_step": round((ms_tot["sdc"] + ms_tot["isdc"]) / 18, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "table1b: 2D viscous Burgers periodic [-1,1)^2 n=128 (h=1/64) Gaussian sigma=0.1 "
                               "WENO5 compact stencil with W dt=1e-3 Lobatto M=3,5,7 nu=0.1,1,10 tol 5e-8; "
                               "SDC inner_tol 1e-9; ISDC L=2 early exit; weighted-Jacobi V(3,3)"},
        "time_savings_pct": round(100.0 * (1 - ms_tot["isdc"] / ms_tot["sdc"]), 2),
        "totals": {"sdc_vcycles": tot["sdc"], "isdc_vcycles": tot["isdc"],
                   "sdc_ms": round(ms_tot["sdc"], 3), "isdc_ms": round(ms_tot["isdc"], 3)},
        "printed_savings_pct_9_rows": round(printed_save, 2),
        "rows": rows,
    }


def workload_text(name, cfg):
    return (f"{name}: {cfg['dim']}D n={cfg['n']} {'periodic' if cfg.get('bc', 0) == 1 else 'Dirichlet'} "
            f"nu={cfg['nu']} fe={['zero', 'cubic', 'WENO5 Burgers'][cfg['fe_kind']]} "
            f"{['Lobatto', 'Radau-right', 'Legendre'][cfg['node_kind']]} M={cfg['M']} dt={cfg['dt']} L=2 "
            + ("compact 4th-order stencil with W, " if cfg.get("stencil", 0) == 1 else "")
            + ("Jacobi" if cfg.get("smoother", 0) == 1 else "RBGS")
            + f" V({cfg.get('nu_pre', 1)},{cfg.get('nu_post', 1)})"
            + f" tol={cfg['sdc_tol']}"
            + (" two-level MLSDC (coarse level (n-1)/2, FAS, cubic interpolation)" if cfg.get("levels", 1) == 2 else ""))


def serve_latency(args, torch, count=48):
    """p50 / p99 latency of a short serving run (the serving workload's request
    mix, `count` requests): saturated capacity first (all requests at t = 0),
    then Poisson arrivals at half of it."""
    from paper_1401_7824_amd.serve import Server, make_requests
    budget = int(args.serve_budget_gb * 2 ** 30)

    def server():
        return Server(budget, slots_per_batch=64, precision=1, vcycles=2, solo_workers=args.serve_solo)

    server().serve(make_requests(8, rate=0.0, seed=99))
    sat = server().serve(make_requests(count, rate=0.0, seed=5))
    cap = sat.completed / sat.makespan
    half = server().serve(make_requests(count, rate=0.5 * cap, seed=5)).summary()
    return {"requests": count, "capacity_req_s": round(cap, 3), "rate_req_s": round(0.5 * cap, 3),
            "p50_ms": half["p50_ms"], "p99_ms": half["p99_ms"], "saturated_p50_ms": sat.summary()["p50_ms"],
            "saturated_p99_ms": sat.summary()["p99_ms"], "hbm_budget_gib": args.serve_budget_gb}


def run_followed(args, cfg, torch):
    """Steps/s of a second-order-stencil workload with the dominant kernel's
    duration taken inside the timed steps.  A survey step per followed kernel
    finds the kernel with the most time per step; during the timed steps every
    launch of it records its own dispatch start and end (hipExtLaunchKernelGGL
    with HIP events, on the stream the kernel runs on), and achieved GB/s =
    its average algorithmic bytes / its average duration."""
    import numpy as np
    from paper_1401_7824_amd import workloads as W
    name = args.workload
    T = "double" if cfg["precision"] == 0 else "float"
    plan = make_plan(cfg)
    shapes = plan.autotune()  # tile shape per level (timed once, then cached), outside the timed steps
    modes = W.workload_modes(cfg) if "gaussian_sigma" not in cfg else None
    u = torch.from_numpy(W.workload_u0(cfg)).cuda()
    survey, nsurvey = kernel_survey(plan, u, cfg["dt"], cfg)
    print(f"[bench] {name}: survey of {len(survey)} kernels in {nsurvey} steps done", file=sys.stderr, flush=True)
    dom_key = max(survey, key=lambda k: survey[k][2])
    kind = dict((k, (kd, lv)) for k, kd, lv in PROBE_KINDS)[dom_key]
    for _ in range(args.warmup):
        plan.step(u, cfg["dt"])
    plan.probe_arm(kind[0], kind[1], 1, 1000000)
    elapsed, wall, stats = time_steps(plan, u, cfg["dt"], args.steps, 0, torch)
    nl, avg_us, alg_b = plan.probe_read()
    print(f"[bench] {name}: {args.steps} timed steps in {elapsed:.3f} s", file=sys.stderr, flush=True)
    # as many further steps with no kernel followed: what the per-launch event
    # pairs cost, which shows only where the followed launches are short
    elapsed_free, _, stats_free = time_steps(plan, u, cfg["dt"], args.steps, 0, torch)
    sweeps = sum(s.sweeps for s in stats) / len(stats)
    vcyc = sum(s.vcycles for s in stats) / len(stats)
    kname = probe_kernel_name(dom_key, cfg, T, (shapes or [0])[0])
    gbps = alg_b / (avg_us * 1e-6) / 1e9
    traffic = counter_traffic(kname, name)
    roof = dict(bound="hbm", achieved=round(gbps, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(gbps / HBM_PEAK_GBS, 4), traffic=traffic, kernel=kname + " (finest level)",
                avg_launch_us=round(avg_us, 3), launches_timed=nl, alg_bytes_per_launch=alg_b,
                timing="each launch of the kernel inside the timed steps, its dispatch start/end in HIP events")
    total = sum(v[2] for v in survey.values())
    kernels = {k: dict(kernel=probe_kernel_name(k, cfg, T, (shapes or [0])[0]), launches_per_step=v[0],
                       avg_us=round(v[1], 3), us_per_step=round(v[2], 1), alg_bytes=v[3],
                       gbps=round(v[3] / (v[1] * 1e-6) / 1e9, 1) if v[1] > 0 else None)
               for k, v in sorted(survey.items(), key=lambda kv: -kv[1][2])}
    out = {
        "metric": METRIC, "value": round(args.steps / elapsed, 4), "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if cfg["precision"] == 0 else "f64+f32", "data": "synthetic",
        "config": {"workload": workload_text(name, cfg), "sweeps_per_step": sweeps, "vcycles_per_step": vcyc,
                   "coarse_vcycles_per_step": sum(s.coarse_vcycles for s in stats) / len(stats),
                   "host_wall_s": round(wall, 4), "tile_shapes": shapes,
                   "survey_steps": nsurvey},
        "roofline": roof,
        "kernels_followed_us_per_step": kernels,
        # later steps of the same integration may take other sweep counts, so the
        # time per sweep is the comparable figure
        "unobserved": {"steps_per_s": round(args.steps / elapsed_free, 4),
                       "sweeps_per_step": sum(s.sweeps for s in stats_free) / len(stats_free),
                       "ms_per_sweep": round(elapsed_free * 1e3 / sum(s.sweeps for s in stats_free), 4),
                       "ms_per_sweep_followed": round(elapsed * 1e3 / sum(s.sweeps for s in stats), 4)},
        "kernel_share_of_step": round(total / (elapsed / args.steps * 1e6), 3),
    }
    nstep = nsurvey + args.warmup + 2 * args.steps  # survey, warm-up, followed and unobserved steps
    if cfg["fe_kind"] == W.FE_ZERO and modes is not None:
        ref = collocation_reference(cfg, modes, nstep)
        got = u.cpu().numpy()
        out["accuracy"] = {"rel_l2_vs_collocation": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                           "steps_compared": nstep,
                           "reference": "sine modes of u_0 times R(dt nu lambda)^steps, R the Pade closed form"}
    del plan
    torch.cuda.empty_cache()
    if cfg["precision"] == 0 and name == "heat3d":
        # the float32-V-cycle variant of the same workload (FP64 residual, S*F and update)
        mc = dict(cfg, precision=1)
        mplan = make_plan(mc)
        mshapes = mplan.autotune()
        um = torch.from_numpy(W.workload_u0(mc)).cuda()
        for _ in range(args.warmup):
            mplan.step(um, mc["dt"])
        m_el, _, m_stats = time_steps(mplan, um, mc["dt"], args.steps, 0, torch)
        ref = collocation_reference(mc, modes, args.warmup + args.steps)
        got = um.cpu().numpy()
        out["mixed"] = {"steps_per_s": round(args.steps / m_el, 4), "ms_per_step": round(m_el / args.steps * 1e3, 4),
                        "sweeps_per_step": sum(s.sweeps for s in m_stats) / len(m_stats),
                        "vcycles_per_step": sum(s.vcycles for s in m_stats) / len(m_stats),
                        "rel_l2_vs_collocation": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                        "steps_compared": args.warmup + args.steps, "tile_shapes": mshapes}
        del mplan, um
        torch.cuda.empty_cache()
        print(f"[bench] {name}: mixed variant {out['mixed']['steps_per_s']} steps/s", file=sys.stderr, flush=True)
    if not args.no_serve_latency and name == "heat3d":
        out["latency"] = serve_latency(args, torch)
        print(f"[bench] serving latency {out['latency']}", file=sys.stderr, flush=True)
    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, sweeps)
    return out


COMPARE_VARIANTS = [
    # (name, params): classical SDC solves each implicit system to tol / 50;
    # ISDC runs L = 2 cycles of the given smoother (Sec. 3, Sec. 4.2)
    ("sdc_classical_rbgs11", dict(vcycles=0, smoother=0, nu_pre=1, nu_post=1)),
    ("sdc_classical_jacobi33", dict(vcycles=0, smoother=1, nu_pre=3, nu_post=3)),
    ("isdc_rbgs11", dict(vcycles=2, smoother=0, nu_pre=1, nu_post=1)),
    ("isdc_rbgs22", dict(vcycles=2, smoother=0, nu_pre=2, nu_post=2)),
    ("isdc_jacobi22", dict(vcycles=2, smoother=1, nu_pre=2, nu_post=2)),
    ("isdc_jacobi33", dict(vcycles=2, smoother=1, nu_pre=3, nu_post=3)),
]


def run_compare(args, torch):
    """The paper's comparison (Sec. 4.2, Table 1) at full size: classical SDC
    (every implicit system solved by V-cycles until its max-norm residual
    <= sdc_tol / 50) against ISDC with L = 2 V-cycles per solve and several
    smoothers, on the rd2d and heat3d workloads (all float64).  Every variant
    runs the same first step from u_0 (--steps timed repetitions after one
    untimed one); reports sweeps, V-cycles and time per step."""
    from paper_1401_7824_amd import Plan, workloads as W
    out_rows = {}
    for wname in ("rd2d", "heat3d"):
        cfg = dict(W.WORKLOADS[wname], precision=0)
        u0 = torch.from_numpy(W.workload_u0(cfg)).cuda()
        rows = {}
        for vname, par in COMPARE_VARIANTS:
            p = Plan(cfg["dim"], cfg["n"], cfg["nu"], cfg["fe_kind"], node_kind=cfg["node_kind"], M=cfg["M"],
                     precision=0, sdc_tol=cfg["sdc_tol"], inner_tol=cfg["sdc_tol"] / 50, max_sweeps=200, **par)
            if par["smoother"] == 0:
                p.autotune()
            u = u0.clone()
            st = p.step(u, cfg["dt"])
            reps = max(1, args.steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                u.copy_(u0)
                p.step(u, cfg["dt"])
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / reps * 1e3
            rows[vname] = {"sweeps": st.sweeps, "vcycles": st.vcycles, "status": st.status,
                           "ms_per_step": round(ms, 3)}
            print(f"[compare] {wname} {vname}: {st.sweeps} sweeps, {st.vcycles} V-cycles, {ms:.2f} ms/step",
                  file=sys.stderr, flush=True)
            del p
            torch.cuda.empty_cache()
        out_rows[wname] = rows
    best = min(out_rows["heat3d"].items(), key=lambda kv: kv[1]["ms_per_step"])
    return {
        "metric": "ISDC vs classical SDC at full size: time per step and V-cycles",
        "value": round(1e3 / best[1]["ms_per_step"], 4), "unit": "steps/s", "n_gpus": 1,
        "steps": max(1, args.steps) * len(COMPARE_VARIANTS) * 2, "warmup": len(COMPARE_VARIANTS) * 2,
        "ms_per_step": best[1]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "compare: rd2d 1023^2 Lobatto M=5 and heat3d 255^3 Radau-right M=3, first step "
                               "from u_0, tol 1e-10; classical SDC inner tolerance 2e-12",
                   "fastest_heat3d_variant": best[0]},
        "rows": out_rows,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); runs on several GPUs are not supported",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1401_7824_amd as P
    from paper_1401_7824_amd import workloads as W
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    P.load()
    if args.workload == "batch":
        print(json.dumps(run_batch(args, torch)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args, torch)), flush=True)
        return
    if args.workload == "table1":
        print(json.dumps(run_table1(args, torch)), flush=True)
        return
    if args.workload == "table1b":
        print(json.dumps(run_table1b(args, torch)), flush=True)
        return
    if args.workload == "compare":
        print(json.dumps(run_compare(args, torch)), flush=True)
        return
    if args.workload == "kernels":
        print(json.dumps(run_kernels(args, torch)), flush=True)
        return
    cfg = dict(W.WORKLOADS[args.workload])
    if cfg.get("stencil", 0) == 0:
        print(json.dumps(run_followed(args, cfg, torch)), flush=True)
        return
    plan = make_plan(cfg)
    shapes = plan.autotune()  # tile shape per level (timed once, then cached), outside the timed steps
    u = torch.from_numpy(W.workload_u0(cfg)).cuda()
    accuracy = None
    if cfg["fe_kind"] == W.FE_ZERO and cfg.get("bc", 0) == 0:
        accuracy = accuracy_vs_collocation(cfg, torch)
    elapsed, wall, stats = time_steps(plan, u, cfg["dt"], args.steps, args.warmup, torch)
    sweeps = sum(s.sweeps for s in stats) / len(stats)
    vcyc = sum(s.vcycles for s in stats) / len(stats)
    kp = kernel_probe(plan, cfg, args.probe_reps, torch)
    vc = vcycle_probe(plan, cfg, 20, torch)
    dom = kp.get("smooth_restrict") or kp.get("prolong_smooth") or kp.get("smooth") or kp["tail"]
    traffic = counter_traffic(dom["kernel"], args.workload)
    roof = dict(bound="hbm", achieved=dom["gbps"], peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(dom["gbps"] / HBM_PEAK_GBS, 4), traffic=traffic, kernel=dom["kernel"] + " (finest level)",
                avg_launch_us=dom["avg_us"], alg_bytes_per_launch=dom["alg_bytes"])
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
        "config": {"workload": f"{args.workload}: {cfg['dim']}D n={cfg['n']} "
                               f"{'periodic' if cfg.get('bc', 0) == 1 else 'Dirichlet'} nu={cfg['nu']} "
                               f"fe={['zero', 'cubic', 'WENO5 Burgers'][cfg['fe_kind']]} "
                               f"{'Lobatto' if cfg['node_kind'] == 0 else 'Radau-right'} M={cfg['M']} "
                               f"dt={cfg['dt']} L=2 "
                               + ("compact 4th-order stencil with W, Jacobi "
                                  f"V({cfg.get('nu_pre')},{cfg.get('nu_post')})" if cfg.get("stencil", 0) == 1
                                  else "RBGS V(1,1)") + f" tol={cfg['sdc_tol']}"
                               + (" two-level MLSDC (511^2 coarse level, FAS, cubic interpolation)"
                                  if cfg.get("levels", 1) == 2 else ""),
                   "sweeps_per_step": sweeps, "vcycles_per_step": vcyc,
                   "coarse_vcycles_per_step": sum(s.coarse_vcycles for s in stats) / len(stats),
                   "host_wall_s": round(wall, 4), "tile_shapes": shapes},
        "roofline": roof,
        "vcycle": vc,
        "kernels": kp,
    }
    if accuracy is not None:
        out["accuracy"] = accuracy
    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, sweeps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
