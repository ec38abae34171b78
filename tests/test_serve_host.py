"""Host-side checks of the request generator of the serving loop (no GPU)."""

import numpy as np

from paper_1401_7824_amd.serve import make_requests


def test_request_mix_and_poisson_arrivals():
    reqs = make_requests(400, rate=50.0, seed=5, big=False)
    dims = np.array([r.dim for r in reqs])
    assert 0.35 < (dims == 2).mean() < 0.65
    assert all(r.n in (127, 255) for r in reqs if r.dim == 2)
    assert all(r.n in (31, 63) for r in reqs if r.dim == 3)
    assert {r.sdc_tol for r in reqs} == {1e-5, 1e-8}
    assert {r.M for r in reqs} == {3, 5}
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert np.all(gaps >= 0)
    assert 0.015 < gaps.mean() < 0.025  # mean inter-arrival 1/rate
    again = make_requests(400, rate=50.0, seed=5, big=False)
    assert all(np.array_equal(a.u0, b.u0) and a.arrival == b.arrival for a, b in zip(reqs, again))


def test_all_at_once_when_rate_is_zero():
    reqs = make_requests(10, rate=0.0, seed=1, big=False)
    assert all(r.arrival == 0.0 for r in reqs)


class _Req:
    def __init__(self, rid, dim, size):
        self.rid, self.dim, self.size = rid, dim, size


def test_admission_first_come_first_served_with_reservation():
    from paper_1401_7824_amd.serve import choose_admissions
    need = lambda r: r.size  # noqa: E731
    w = [_Req(0, 2, 4), _Req(1, 3, 8), _Req(2, 2, 1), _Req(3, 3, 1)]
    # 10 bytes: 0 fits; 1 does not (4 + 8 > 10) and reserves 8: 2 and 3 must fit beside it, 4 + 8 + 1 > 10
    got = choose_admissions(w, need, 0, 10, {2: 4, 3: 4})
    assert [r.rid for r in got] == [0]
    # with 14 bytes: 0, 1, then 2 and 3 (4 + 8 + 1 + 1 = 14)
    assert [r.rid for r in choose_admissions(w, need, 0, 14, {2: 4, 3: 4})] == [0, 1, 2, 3]
    # no free slot in 3D: request 1 waits for a slot and reserves its memory; 2D requests behind it still run
    assert [r.rid for r in choose_admissions(w, need, 0, 14, {2: 4, 3: 0})] == [0, 2]
    assert choose_admissions([], need, 0, 14, {2: 4}) == []


def test_large_request_is_not_starved_by_steady_small_arrivals():
    # Fake clock: one small request arrives every tick and runs for 3 ticks; a
    # large request needing most of the budget arrives at tick 5.  Without the
    # reservation the small ones would keep the memory busy for ever; with it
    # the large request is admitted as soon as the running small ones drain.
    from paper_1401_7824_amd.serve import choose_admissions
    budget, small, large = 10, 3, 8
    need = lambda r: r.size  # noqa: E731
    waiting, running = [], []  # running: (request, finish tick)
    admitted_at = {}
    rid = 0
    for tick in range(60):
        running = [(r, t) for r, t in running if t > tick]
        waiting.append(_Req(rid, 2, small))
        rid += 1
        if tick == 5:
            waiting.append(_Req(-1, 3, large))
        used = sum(r.size for r, _ in running)
        for r in choose_admissions(waiting, need, used, budget, {2: 64, 3: 64}):
            admitted_at[r.rid] = tick
            running.append((r, tick + 3))
            waiting.remove(r)
    assert -1 in admitted_at
    assert admitted_at[-1] <= 5 + 3  # the running small requests finish within 3 ticks


def test_2d_requests_run_weighted_jacobi_cycles_3d_red_black():
    from paper_1401_7824_amd import _capi as A
    from paper_1401_7824_amd.serve import Request, runs_solo
    big = Request(rid=0, dim=2, n=511, nu=0.1, fe_kind=1, modes=[], dt=1e-3, nsteps=1, sdc_tol=1e-8)
    small = Request(rid=1, dim=2, n=127, nu=1.0, fe_kind=0, modes=[], dt=1e-3, nsteps=1, sdc_tol=1e-8)
    cube = Request(rid=2, dim=3, n=127, nu=1.0, fe_kind=0, modes=[], dt=1e-3, nsteps=1, sdc_tol=1e-8)
    assert runs_solo(big, 5) and runs_solo(cube, 5) and not runs_solo(small, 5) and runs_solo(small, 0)
    for r in (big, small):
        p = r.params(1, 2)
        assert (p["smoother"], p["nu_pre"], p["nu_post"]) == (A.SMOOTH_JACOBI, 3, 3)
    assert "smoother" not in cube.params(1, 2)
