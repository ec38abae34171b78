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
