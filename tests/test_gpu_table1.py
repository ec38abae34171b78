"""Table 1(a) replay on the GPU (Sec. 4): classical SDC against ISDC on the 2D
heat equation, u0 = sin(pi x) sin(pi y), h = 1/64, dt = 1e-3, Gauss-Lobatto
M in {3, 5, 7}, nu in {1, 10, 100}, sweeps until the max-norm SDC residual is
below 5e-8.  Classical SDC cycles every implicit solve until its max-norm
residual is at most 1e-9; ISDC stops after L = 2 cycles, or earlier once that
tolerance is met.  Two multigrid settings: weighted-Jacobi V(3,3) (the one
the replay reports) and the default red-black Gauss-Seidel V(1,1).

The accumulated V-cycle and sweep counts of the GPU path must equal the
oracle's, and the final states must agree to 1e-12.  The printed counts come
from the paper's own multigrid (fourth-order compact stencil, a solver it does
not specify) and are not reproduced; only the qualitative statements of Sec. 4
are asserted: ISDC never needs fewer sweeps than SDC, and with a solver that
needs at most two cycles per solve the two methods coincide."""

import numpy as np
import pytest

import oracle as O
from oracle.sdc import SDCConfig, sdc_step
from gpu_helpers import announce, dev, host, require_gpu

pytestmark = pytest.mark.gpu

N, DT, TOL, INNER = 63, 1e-3, 5e-8, 1e-9
ROWS = [(nu, M) for nu in (1.0, 10.0, 100.0) for M in (3, 5, 7)]
MG = {"jac33": dict(smoother=O.SMOOTH_JACOBI, nu1=3, nu2=3), "rbgs11": dict(smoother=O.SMOOTH_RBGS, nu1=1, nu2=1)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _u0():
    x = np.arange(1, N + 1) / (N + 1)
    return np.outer(np.sin(np.pi * x), np.sin(np.pi * x))


def _mode(isdc):
    return dict(vcycles=2, early_exit=True) if isdc else dict(vcycles=0, early_exit=False)


def _gpu_step(nu, M, isdc, u0, mg="jac33"):
    from paper_1401_7824_amd import Plan
    g = MG[mg]
    p = Plan(2, N, nu, O.FE_ZERO, node_kind=O.NODES_LOBATTO, M=M, sdc_tol=TOL, inner_tol=INNER,
             max_sweeps=100, smoother=g["smoother"], nu_pre=g["nu1"], nu_post=g["nu2"], **_mode(isdc))
    u = dev(u0)
    st = p.step(u, DT)
    return host(u), st


def _oracle_step(nu, M, isdc, u0, mg="jac33"):
    cfg = SDCConfig(nu=nu, node_kind=O.NODES_LOBATTO, M=M, inner="mg", tol=TOL, inner_tol=INNER,
                    max_sweeps=100, **MG[mg], **_mode(isdc))
    return sdc_step(u0, DT, 1.0 / (N + 1), cfg)


@pytest.mark.parametrize("mg", list(MG))
@pytest.mark.parametrize("isdc", [False, True], ids=["sdc", "isdc"])
@pytest.mark.parametrize("nu,M", ROWS)
def test_table1_counts_equal_oracle(nu, M, isdc, mg):
    announce("table1", nu, M, "isdc" if isdc else "sdc", mg)
    u0 = _u0()
    got, st = _gpu_step(nu, M, isdc, u0, mg)
    ref, rst = _oracle_step(nu, M, isdc, u0, mg)
    assert st.status == "ok" and rst.status == "ok"
    assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("nu,M", ROWS)
def test_isdc_needs_at_least_the_sdc_sweeps(nu, M):
    announce("table1 sweeps", nu, M)
    u0 = _u0()
    _, s = _gpu_step(nu, M, False, u0)
    _, i = _gpu_step(nu, M, True, u0)
    assert i.sweeps >= s.sweeps


def test_sdc_reduces_to_isdc_when_solves_are_cheap():
    # nu = 0.1 (diffusive CFL 0.41, the mildest setting of Sec. 4): from the
    # warm start every classical solve meets the tolerance within two cycles,
    # so the early-exit ISDC run makes exactly the same cycles and sweeps
    announce("table1 non-stiff")
    u0 = _u0()
    gs, s = _gpu_step(0.1, 3, False, u0)
    gi, i = _gpu_step(0.1, 3, True, u0)
    assert (s.sweeps, s.vcycles) == (i.sweeps, i.vcycles) == (2, 6)
    assert np.array_equal(gs, gi)
