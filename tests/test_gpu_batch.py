"""Batched ISDC on the GPU: every slot's result must be bitwise the result of
the same instance run alone with isdc_step (same kernel bodies, same
coefficients), whatever else shares the batch, whenever it joins, and even
when a neighbour fails."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

LOB, RAD = O.NODES_LOBATTO, O.NODES_RADAU_RIGHT


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _alone(d, n, nu, fe, u0, dt, nsteps, **par):
    from paper_1401_7824_amd import Plan
    p = Plan(d, n, nu, fe, **par)
    u = dev(u0)
    stats = [p.step(u, dt) for _ in range(nsteps)]
    return host(u), stats


def _instances(d, prec, count, seed):
    rng = np.random.default_rng(seed)
    sizes = {1: [127, 1023, 4095], 2: [31, 63, 127, 255], 3: [15, 31, 63]}[d]
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        M = int(rng.choice([3, 5]))
        kind = LOB if rng.random() < 0.7 else RAD
        fe = O.FE_CUBIC if rng.random() < 0.5 else O.FE_ZERO
        nu = float(rng.uniform(0.05, 1.0))
        dt = float(rng.uniform(2e-4, 5e-3))
        u0 = 2.0 * W.sine_field(n, d, W.draw_modes(d, 6, seed=seed * 100 + i, max_wave=8 if d == 1 else 4))
        out.append(dict(d=d, n=n, nu=nu, fe=fe, dt=dt, u0=u0,
                        par=dict(node_kind=kind, M=M, precision=prec, sdc_tol=1e-10 if prec == 0 else 1e-9)))
    return out


@pytest.mark.parametrize("d,prec", [(2, 0), (2, 1), (1, 0), (3, 1)])
def test_batch_slots_equal_single_instance_runs(d, prec):
    from paper_1401_7824_amd import Batch
    announce("batch equal", d, prec)
    inst = _instances(d, prec, 7, seed=10 + d + 4 * prec)
    b = Batch(8, d, precision=prec, vcycles=2)
    us = []
    for i, x in enumerate(inst):
        u = dev(x["u0"])
        b.set(i, u, x["dt"], 2, x["nu"], x["fe"], **x["par"])
        us.append(u)
    b.run()
    for i, x in enumerate(inst):
        state, status, steps, st = b.info(i)
        ref, rstats = _alone(d, x["n"], x["nu"], x["fe"], x["u0"], x["dt"], 2, **x["par"])
        assert status == "ok" and steps == 2, (i, status)
        assert np.array_equal(host(us[i]), ref), f"slot {i} differs from the single-instance run"
        assert st.sweeps == rstats[-1].sweeps and st.vcycles == rstats[-1].vcycles


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_marched_3d_slots_equal_single_instance_runs(prec):
    # 127^3 levels run the z-marched kernels (float32 and float64 plane
    # layouts differ in tile height); slots still equal the plan's bits
    from paper_1401_7824_amd import Batch
    announce("batch marched 3d", prec)
    d, n = 3, 127
    inst = []
    for i, (nu, fe, dt) in enumerate([(0.3, O.FE_CUBIC, 2e-3), (1.0, O.FE_ZERO, 1e-3)]):
        u0 = 2.0 * W.sine_field(n, d, W.draw_modes(d, 6, seed=900 + i, max_wave=4))
        inst.append(dict(nu=nu, fe=fe, dt=dt, u0=u0,
                         par=dict(node_kind=LOB, M=3, precision=prec, sdc_tol=1e-10 if prec == 0 else 1e-9)))
    b = Batch(2, d, precision=prec, vcycles=2)
    us = []
    for i, x in enumerate(inst):
        u = dev(x["u0"])
        b.set(i, u, x["dt"], 1, x["nu"], x["fe"], **x["par"])
        us.append(u)
    b.run()
    for i, x in enumerate(inst):
        state, status, steps, st = b.info(i)
        ref, rstats = _alone(d, n, x["nu"], x["fe"], x["u0"], x["dt"], 1, **x["par"])
        assert status == "ok" and steps == 1, (i, status)
        assert np.array_equal(host(us[i]), ref), f"slot {i} differs from the single-instance run"
        assert st.sweeps == rstats[-1].sweeps and st.vcycles == rstats[-1].vcycles


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_255_cube_slot_equals_single_instance_run(prec):
    # the benchmark's grid: 255^3 and its 127^3 level run the z-marched
    # kernels, the fused smoothing + restriction with its fitted column depth
    # (six columns a tile on 255^3) in the plan, the separate kernels in the
    # batch; Radau-right M = 3 heat, the benchmark's node set
    from paper_1401_7824_amd import Batch
    announce("batch 255^3", prec)
    d, n, nu, dt = 3, 255, 1.0, 1e-3
    u0 = W.sine_field(n, d, W.draw_modes(d, 8, seed=4242, max_wave=4))
    par = dict(node_kind=RAD, M=3, precision=prec, sdc_tol=1e-10 if prec == 0 else 1e-9)
    b = Batch(1, d, precision=prec, vcycles=2)
    u = dev(u0)
    b.set(0, u, dt, 1, nu, O.FE_ZERO, **par)
    b.run()
    state, status, steps, st = b.info(0)
    ref, rstats = _alone(d, n, nu, O.FE_ZERO, u0, dt, 1, **par)
    assert status == "ok" and steps == 1, status
    assert np.array_equal(host(u), ref), "the 255^3 slot differs from the single-instance run"
    assert st.sweeps == rstats[-1].sweeps and st.vcycles == rstats[-1].vcycles


def test_continuous_batching_join_and_leave():
    # slots join while others are mid-step and a finished slot is reused;
    # every result equals its run alone
    from paper_1401_7824_amd import Batch
    announce("batch continuous")
    inst = _instances(2, 0, 6, seed=31)
    b = Batch(3, 2, precision=0, vcycles=2)
    us = {}
    pending = list(range(len(inst)))
    done = []
    free = [0, 1, 2]
    where = {}
    sweeps = 0
    while pending or any(s is not None for s in where.values()):
        while free and pending:
            k = pending.pop(0)
            slot = free.pop(0)
            x = inst[k]
            u = dev(x["u0"])
            b.set(slot, u, x["dt"], 1 + k % 2, x["nu"], x["fe"], **x["par"])
            us[k] = u
            where[slot] = k
        b.advance()
        sweeps += 1
        for slot, k in list(where.items()):
            if k is None:
                continue
            state, status, steps, _ = b.info(slot)
            if state == 2:
                assert status == "ok"
                done.append(k)
                b.release(slot)
                where[slot] = None
                free.append(slot)
        assert sweeps < 5000
    assert sorted(done) == list(range(len(inst)))
    for k, x in enumerate(inst):
        ref, _ = _alone(2, x["n"], x["nu"], x["fe"], x["u0"], x["dt"], 1 + k % 2, **x["par"])
        assert np.array_equal(host(us[k]), ref), f"instance {k}"


def test_failing_slot_does_not_disturb_neighbours():
    from paper_1401_7824_amd import Batch
    announce("batch failure isolation")
    inst = _instances(2, 0, 3, seed=41)
    bad = inst[1]["u0"].copy()
    bad[3, 4] = np.nan
    inst[1]["u0"] = bad
    inst[2]["par"]["max_sweeps"] = 2
    inst[2]["par"]["sdc_tol"] = 1e-15
    b = Batch(3, 2, precision=0, vcycles=2)
    us = []
    for i, x in enumerate(inst):
        u = dev(x["u0"])
        b.set(i, u, x["dt"], 1, x["nu"], x["fe"], **x["par"])
        us.append(u)
    b.run()
    assert b.info(0)[1] == "ok"
    assert b.info(1)[1] == "diverged"
    assert b.info(2)[1] == "not_converged" and b.info(2)[3].sweeps == 2
    ref0, _ = _alone(2, inst[0]["n"], inst[0]["nu"], inst[0]["fe"], inst[0]["u0"], inst[0]["dt"], 1, **inst[0]["par"])
    assert np.array_equal(host(us[0]), ref0)
    ref2, _ = _alone(2, inst[2]["n"], inst[2]["nu"], inst[2]["fe"], inst[2]["u0"], inst[2]["dt"], 1, **inst[2]["par"])
    assert np.array_equal(host(us[2]), ref2)


def test_batch_matches_oracle_collocation():
    # a batched heat instance also lands on the direct collocation solution
    from paper_1401_7824_amd import Batch
    announce("batch vs collocation")
    n, nu, dt = 127, 0.5, 2e-3
    u0 = W.sine_field(n, 2, W.draw_modes(2, 8, seed=5))
    b = Batch(2, 2, precision=1, vcycles=2)
    u = dev(u0)
    b.set(0, u, dt, 1, nu, O.FE_ZERO, node_kind=LOB, M=5, sdc_tol=1e-11)
    b.run()
    coll = O.collocation_heat_modal(u0, dt, nu, 1.0 / (n + 1), LOB, 5)
    got = host(u)
    assert np.linalg.norm(got - coll) / np.linalg.norm(coll) < 1e-8


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_jacobi_2d_slots_equal_single_instance_runs(prec):
    # 2D weighted-Jacobi slots (V(3,3) and V(2,1): the fused row kernels with
    # 3, 2 and 1 steps) beside red-black V(1,1) slots in one batch; every slot
    # equals its run alone bit for bit
    from paper_1401_7824_amd import Batch
    announce("batch jacobi 2d", prec)
    inst = _instances(2, prec, 9, seed=70 + prec)
    cycles = [dict(smoother=1, nu_pre=3, nu_post=3), dict(smoother=1, nu_pre=2, nu_post=1), dict()]
    b = Batch(9, 2, precision=prec, vcycles=2)
    us = []
    for i, x in enumerate(inst):
        x["par"].update(cycles[i % 3])
        u = dev(x["u0"])
        b.set(i, u, x["dt"], 2, x["nu"], x["fe"], **x["par"])
        us.append(u)
    b.run()
    for i, x in enumerate(inst):
        state, status, steps, st = b.info(i)
        ref, rstats = _alone(2, x["n"], x["nu"], x["fe"], x["u0"], x["dt"], 2, **x["par"])
        assert status == "ok" and steps == 2, (i, status)
        assert np.array_equal(host(us[i]), ref), f"slot {i} ({cycles[i % 3]}) differs from the single-instance run"
        assert st.sweeps == rstats[-1].sweeps and st.vcycles == rstats[-1].vcycles


def test_batch_rejects_unsupported_parameters():
    from paper_1401_7824_amd import Batch, ISDCError
    announce("batch unsupported")
    b = Batch(2, 2, precision=0, vcycles=2)
    u = dev(np.zeros((31, 31)))
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, smoother=1, nu_pre=4, nu_post=4)
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, guess=1)
    with pytest.raises(ISDCError):
        b.set(0, u, 1e-3, 1, 1.0, precision=1)  # batch is FP64
    with pytest.raises(ISDCError):
        b.set(5, u, 1e-3, 1, 1.0)  # slot out of range


@pytest.mark.parametrize("d,prec", [(2, 1), (3, 0)])
def test_fixed_batch_step_equals_isdc_step(d, prec):
    # isdc_batch_create / isdc_batch_step: one full step of every active
    # instance per call; instance i is bitwise isdc_step on its own plan
    from paper_1401_7824_amd import FixedBatch, Plan
    announce("fixed batch step", d, prec)
    inst = _instances(d, prec, 5, seed=70 + d + prec)
    fb = FixedBatch(d, [dict(n=x["n"], nu=x["nu"], fe_kind=x["fe"], vcycles=2, **x["par"]) for x in inst])
    us = [dev(x["u0"]) for x in inst]
    refs = [dev(x["u0"]) for x in inst]
    plans = [Plan(d, x["n"], x["nu"], x["fe"], vcycles=2, **x["par"]) for x in inst]
    masks = [None, [True, False, True, True, False]]
    for call, active in enumerate(masks):
        status, stats = fb.step(us, [x["dt"] for x in inst], active)
        assert status == "ok"
        for i, x in enumerate(inst):
            if active is not None and not active[i]:
                assert stats[i] is None
                continue
            st = plans[i].step(refs[i], x["dt"])
            assert torch.equal(us[i], refs[i]), f"call {call}: instance {i} differs from isdc_step"
            assert (stats[i].sweeps, stats[i].vcycles) == (st.sweeps, st.vcycles)
            assert stats[i].residual_hist == st.residual_hist
    # inactive instances kept their state: one step behind the others
    for i in (1, 4):
        ref = dev(inst[i]["u0"])
        plans[i].step(ref, inst[i]["dt"])
        assert torch.equal(us[i], ref)


def test_sweep_schedule_timing_eager_and_graph_then_slots_still_exact():
    # isdc_batch_time_sweeps replays the sweep's launches (eager or from one
    # captured HIP graph) for timing; re-set slots afterwards give isdc_step's bits
    from paper_1401_7824_amd import Batch
    announce("batch sweep timing")
    d, prec = 2, 1
    inst = _instances(d, prec, 4, seed=55)
    b = Batch(4, d, precision=prec, vcycles=2)
    side = torch.cuda.Stream()
    us = [dev(x["u0"]) for x in inst]
    for i, x in enumerate(inst):
        b.set(i, us[i], x["dt"], 1, x["nu"], x["fe"], **x["par"])
    torch.cuda.synchronize()
    b.advance(side)
    t_eager, n_eager = b.time_sweeps(3, False, side)
    t_graph, n_graph = b.time_sweeps(3, True, side)
    assert t_eager > 0 and t_graph > 0 and n_eager == n_graph > 10
    for i in range(4):
        b.release(i)
    us = [dev(x["u0"]) for x in inst]
    for i, x in enumerate(inst):
        b.set(i, us[i], x["dt"], 1, x["nu"], x["fe"], **x["par"])
    b.run()
    for i, x in enumerate(inst):
        ref, _ = _alone(d, x["n"], x["nu"], x["fe"], x["u0"], x["dt"], 1, **x["par"])
        assert np.array_equal(host(us[i]), ref)
