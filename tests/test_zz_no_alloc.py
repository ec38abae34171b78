"""isdc_step_noalloc (the step on the library's static device scratch) against
isdc_step on a plan with a torch workspace: same kernels, so the same bits,
on two calls in a row, the second on a smaller problem (the scratch keeps the
first call's contents)."""

import ctypes as C

import numpy as np
import pytest
import torch

import oracle as O
from paper_1401_7824_amd import _capi as A
from paper_1401_7824_amd import workloads as W
from gpu_helpers import announce, dev, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


CASES = [
    # (name, d, n, nu, fe, dt, params); the second case is the smaller one
    ("rd2d-255-lob5-fp64", 2, 255, 0.1, O.FE_CUBIC, 1e-3, dict(node_kind=O.NODES_LOBATTO, M=5)),
    ("heat3d-31-rad3-mixed", 3, 31, 1.0, O.FE_ZERO, 1e-3, dict(node_kind=O.NODES_RADAU_RIGHT, M=3, precision=1)),
]


def _via_cabi(d, n, nu, fe, u, dt, **par):
    from paper_1401_7824_amd.isdc import make_params
    lib = A.load()
    prob = A.problem(d, n, nu, fe)
    params = make_params(**par)
    st = A.Stats()
    rc = lib.isdc_step_noalloc(C.byref(prob), C.byref(params), C.c_void_p(u.data_ptr()), dt,
                               C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(st))
    return rc, st


def test_noalloc_step_equals_isdc_step_twice():
    from paper_1401_7824_amd import Plan
    for name, d, n, nu, fe, dt, par in CASES:
        announce("noalloc", name)
        u0 = 2.0 * W.sine_field(n, d, W.draw_modes(d, 8, seed=31 + d))
        u = dev(u0)
        rc, st = _via_cabi(d, n, nu, fe, u, dt, **par)
        assert rc == A.OK, A.load().isdc_last_error()
        ref = dev(u0)
        rst = Plan(d, n, nu, fe, **par).step(ref, dt)
        torch.cuda.synchronize()
        assert torch.equal(u, ref), name
        assert (st.sweeps, st.vcycles) == (rst.sweeps, rst.vcycles)
        assert [st.residual_hist[i] for i in range(st.hist_len)] == rst.residual_hist
        # a second step continues from the first one's result
        rc, st2 = _via_cabi(d, n, nu, fe, u, dt, **par)
        rst2 = Plan(d, n, nu, fe, **par).step(ref, dt)
        assert rc == A.OK and torch.equal(u, ref) and st2.sweeps == rst2.sweeps
    assert np.isfinite(u.double().sum().item())
