"""Host-side checks of the C ABI (no GPU): symbols, struct layout, tables,
workspace sizing and argument validation."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1401_7824_amd import _capi as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isdc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isdc_[a-z_]+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = A.load()
    declared = _declared_functions()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in include/isdc.h but not exported"
    # the binding declares exactly the header's functions
    assert sorted(n for n, _, _ in A.SIGNATURES) == declared


def test_struct_sizes_match():
    lib = A.load()
    s = [C.c_size_t() for _ in range(3)]
    assert lib.isdc_abi_sizes(*[C.byref(x) for x in s]) == 0
    assert [x.value for x in s] == [C.sizeof(A.Problem), C.sizeof(A.Params), C.sizeof(A.Stats)]


@pytest.mark.parametrize("kind,Ms", [(A.NODES_LOBATTO, range(2, 10)), (A.NODES_RADAU_RIGHT, range(1, 10)),
                                     (A.NODES_LEGENDRE, range(1, 10))])
def test_tables_match_oracle(kind, Ms):
    from paper_1401_7824_amd.isdc import tables, end_weights
    for M in Ms:
        tau, Q, S = (np.array(v) for v in tables(kind, M))
        tol = 1e-15 if M <= 7 else 2e-15
        np.testing.assert_allclose(tau, O.nodes(kind, M), atol=1e-16, rtol=0)
        np.testing.assert_allclose(Q, O.qmatrix(kind, M), atol=tol, rtol=0)
        np.testing.assert_allclose(S, O.smatrix(kind, M), atol=tol, rtol=0)
        np.testing.assert_allclose(np.array(end_weights(kind, M)), O.end_weights(kind, M), atol=tol, rtol=0)


def test_tables_reject_bad_arguments():
    lib = A.load()
    buf = (C.c_double * 100)()
    assert lib.isdc_tables(A.NODES_LOBATTO, 1, buf, buf, buf) == A.E_INVAL
    assert lib.isdc_tables(A.NODES_RADAU_RIGHT, 0, buf, buf, buf) == A.E_INVAL
    assert lib.isdc_tables(A.NODES_LOBATTO, 10, buf, buf, buf) == A.E_INVAL
    assert lib.isdc_tables(7, 3, buf, buf, buf) == A.E_INVAL
    assert b"node_kind" in lib.isdc_last_error()
    assert lib.isdc_tables(A.NODES_LEGENDRE, 0, buf, buf, buf) == A.E_INVAL
    assert lib.isdc_tables(A.NODES_LEGENDRE, 10, buf, buf, buf) == A.E_INVAL
    assert lib.isdc_end_weights(A.NODES_LEGENDRE, 10, buf) == A.E_INVAL
    assert lib.isdc_end_weights(A.NODES_LEGENDRE, 3, None) == A.E_INVAL
    assert lib.isdc_end_weights(A.NODES_LEGENDRE, 3, buf) == A.OK


def _params(**kw):
    from paper_1401_7824_amd.isdc import make_params
    return make_params(**kw)


def _bytes(dim, n, nu=1.0, fe=A.FE_ZERO, **kw):
    lib = A.load()
    out = C.c_size_t()
    rc = lib.isdc_workspace_bytes(C.byref(A.problem(dim, n, nu, fe)), C.byref(_params(**kw)), C.byref(out))
    return rc, out.value


def test_default_params():
    p = _params()
    assert (p.node_kind, p.M, p.vcycles, p.smoother, p.nu_pre, p.nu_post, p.precision, p.guess) == \
        (A.NODES_LOBATTO, 3, 2, A.SMOOTH_RBGS, 1, 1, A.PREC_FP64, A.GUESS_PREV_SWEEP)
    assert p.sdc_tol == 1e-10 and p.max_sweeps == 100


def test_workspace_bytes_scale_with_problem():
    rc, b2 = _bytes(2, 1023, M=5)
    assert rc == 0
    N = 1023 ** 2
    # 2(M-1) node arrays + (M-1) S*F arrays (Lobatto) + 3 fine MG arrays, float64
    assert b2 >= (2 * 4 + 4 + 3) * N * 8
    assert b2 < (2 * 4 + 4 + 3) * N * 8 * 1.4
    rc, b3 = _bytes(3, 255, node_kind=A.NODES_RADAU_RIGHT, M=3)
    assert rc == 0 and b3 > (2 * 3 + 3 + 3) * 255 ** 3 * 8
    rc, b1 = _bytes(1, 127)
    assert rc == 0 and b1 < 64 * 1024


@pytest.mark.parametrize("bad", [
    dict(dim=0), dict(dim=4), dict(n=0), dict(n=10), dict(n=16383, dim=2), dict(n=2047, dim=3), dict(nu=-1.0),
    dict(nu=float("nan")), dict(fe=5), dict(M=1), dict(M=10), dict(node_kind=3), dict(vcycles=-1),
    dict(sdc_tol=-1.0), dict(sdc_tol=0.0), dict(sdc_tol=float("inf")), dict(max_sweeps=0), dict(smoother=2), dict(nu_pre=0, nu_post=0),
    dict(nu_pre=9), dict(precision=2), dict(guess=3), dict(early_exit=2), dict(inner_tol=float("nan")),
    dict(levels=0), dict(levels=3), dict(levels=2, n=1),
])
def test_validation_rejects(bad):
    kw = dict(dim=2, n=63, nu=1.0, fe=A.FE_ZERO)
    kw.update({k: v for k, v in bad.items() if k in kw})
    par = {k: v for k, v in bad.items() if k not in ("dim", "n", "nu", "fe")}
    rc, _ = _bytes(kw["dim"], kw["n"], kw["nu"], kw["fe"], **par)
    assert rc == A.E_INVAL
    assert A.load().isdc_last_error() != b""


def test_axis_counts():
    # n[a] = 1 beyond dim; unequal counts on the used axes are a valid grid the library does not run
    lib = A.load()
    out = C.c_size_t()
    par = _params()
    for dim, n, rc in [(2, (63, 63, 1), 0), (3, (31, 31, 31), 0), (1, (127, 1, 1), 0),
                       (2, (63, 63, 3), A.E_INVAL), (1, (127, 127, 1), A.E_INVAL),
                       (2, (63, 31, 1), A.E_UNSUPPORTED), (3, (31, 31, 15), A.E_UNSUPPORTED)]:
        prob = A.Problem(dim=dim, n=(C.c_int32 * 3)(*n), nu=1.0, fe_kind=A.FE_ZERO)
        assert lib.isdc_workspace_bytes(C.byref(prob), C.byref(par), C.byref(out)) == rc, (dim, n)


def _pbytes(dim, n, stencil, bc, fe=A.FE_ZERO, **kw):
    lib = A.load()
    out = C.c_size_t()
    prob = A.problem(dim, n, 1.0, fe, stencil, bc)
    par = _params(**dict(dict(smoother=A.SMOOTH_JACOBI), **kw))
    return lib.isdc_workspace_bytes(C.byref(prob), C.byref(par), C.byref(out)), out.value


def test_periodic_and_burgers_validation():
    SC, S2, BP, BD = A.STENCIL_COMPACT4, A.STENCIL_2ND, A.BC_PERIODIC, A.BC_DIRICHLET
    for n in (4, 128, 8192):
        assert _pbytes(2, n, SC, BP)[0] == 0
        assert _pbytes(2, n, SC, BP, A.FE_BURGERS)[0] == 0
    for n in (2, 3, 31, 127, 16384):  # n = 2^k with 2 <= k <= 13
        assert _pbytes(2, n, SC, BP)[0] == A.E_INVAL
    assert _pbytes(2, 63, SC, 2)[0] == A.E_INVAL  # unknown bc
    assert _pbytes(2, 64, S2, BP)[0] == A.E_UNSUPPORTED  # periodic second-order stencil
    assert _pbytes(3, 64, SC, BP)[0] == A.E_UNSUPPORTED  # compact stencil is 2D
    assert _pbytes(2, 63, SC, BD, A.FE_BURGERS)[0] == A.E_UNSUPPORTED  # Burgers needs periodic
    assert _pbytes(2, 63, S2, BD, A.FE_BURGERS)[0] == A.E_UNSUPPORTED


def test_mlsdc_validation_and_workspace():
    # two-level MLSDC: second-order stencil, Dirichlet; coarse arrays of ((n-1)/2)^d points
    assert _pbytes(2, 64, A.STENCIL_COMPACT4, A.BC_PERIODIC, levels=2)[0] == A.E_UNSUPPORTED
    assert _pbytes(2, 63, A.STENCIL_COMPACT4, A.BC_DIRICHLET, levels=2)[0] == A.E_UNSUPPORTED
    rc1, b1 = _bytes(2, 255, M=3, node_kind=A.NODES_RADAU_RIGHT)
    rc2, b2 = _bytes(2, 255, M=3, node_kind=A.NODES_RADAU_RIGHT, levels=2)
    assert rc1 == 0 and rc2 == 0
    # R U_0..3, U_c 1..3 and S F_c 0..2: 10 coarse arrays of 127^2 doubles, 256-byte aligned
    assert b2 - b1 == 10 * ((127 * 127 * 8 + 255) // 256 * 256)
    rc, b = _bytes(2, 7, levels=2)  # the fine grid fits the tail: the coarse level gets arrays too
    assert rc == 0 and b > _bytes(2, 7)[1]


def test_burgers_workspace_holds_fe_arrays():
    # f^E arrays: u_0 plus 2 (M - 1) node arrays beside the plain periodic plan (Lobatto, M = 3)
    rc0, b0 = _pbytes(2, 256, A.STENCIL_COMPACT4, A.BC_PERIODIC)
    rc1, b1 = _pbytes(2, 256, A.STENCIL_COMPACT4, A.BC_PERIODIC, A.FE_BURGERS)
    assert rc0 == 0 and rc1 == 0
    assert b1 - b0 == (1 + 2 * 2) * 256 * 256 * 8


def test_create_checks_workspace_without_touching_it():
    lib = A.load()
    prob = A.problem(2, 63, 1.0, A.FE_ZERO)
    par = _params()
    need = C.c_size_t()
    assert lib.isdc_workspace_bytes(C.byref(prob), C.byref(par), C.byref(need)) == 0
    h = C.c_void_p()
    fake = C.c_void_p(1 << 40)  # never dereferenced: creation is host-only
    assert lib.isdc_create(C.byref(prob), C.byref(par), fake, need.value - 1, C.byref(h)) == A.E_WORKSPACE
    assert lib.isdc_create(C.byref(prob), C.byref(par), C.c_void_p((1 << 40) + 8), need.value, C.byref(h)) == A.E_WORKSPACE
    assert lib.isdc_create(C.byref(prob), C.byref(par), None, need.value, C.byref(h)) == A.E_WORKSPACE
    assert lib.isdc_create(C.byref(prob), C.byref(par), fake, need.value, C.byref(h)) == 0
    assert h.value
    st = A.Stats()
    assert lib.isdc_get_stats(h, C.byref(st)) == 0 and st.sweeps == 0
    # calls that would need a step in progress are rejected before any device work
    r = C.c_double()
    assert lib.isdc_sweep(h, None, C.byref(r)) == A.E_INVAL
    assert lib.isdc_end(h, fake, None) == A.E_INVAL
    assert lib.isdc_node_values(h, 1, fake, None) == A.E_INVAL
    assert lib.isdc_begin(h, fake, -1.0, None) == A.E_INVAL
    assert lib.isdc_begin(h, fake, float("nan"), None) == A.E_INVAL
    assert lib.isdc_begin(h, None, 1e-3, None) == A.E_INVAL
    assert lib.isdc_step(h, None, 1e-3, None, None) == A.E_INVAL
    assert lib.isdc_vcycle(h, -1.0, A.PREC_FP64, fake, fake, 1, None, None) == A.E_INVAL
    assert lib.isdc_vcycle(h, 1.0, 5, fake, fake, 1, None, None) == A.E_INVAL
    assert lib.isdc_mg_op(h, 99, 0, 1.0, A.PREC_FP64, fake, fake, fake, None, None) == A.E_INVAL
    assert lib.isdc_mg_op(h, A.OP_SMOOTH, 9, 1.0, A.PREC_FP64, fake, fake, fake, None, None) == A.E_INVAL
    lib.isdc_destroy(h)
    lib.isdc_destroy(None)


def test_null_plan_rejected():
    lib = A.load()
    r = C.c_double()
    assert lib.isdc_sweep(None, None, C.byref(r)) == A.E_INVAL
    assert lib.isdc_get_stats(None, C.byref(A.Stats())) == A.E_INVAL


def test_fixed_batch_validation_host_only():
    # isdc_batch_bytes / isdc_batch_create check every instance before any
    # device work; isdc_batch_step rejects NULL states and bad steps first
    lib = A.load()
    from paper_1401_7824_amd.isdc import make_params
    probs = (A.Problem * 3)(A.problem(2, 63, 1.0), A.problem(2, 127, 0.5, A.FE_CUBIC), A.problem(2, 31, 0.1))
    pars = (A.Params * 3)(make_params(precision=1), make_params(precision=1, M=5), make_params(precision=1))
    out = C.c_size_t()
    assert lib.isdc_batch_bytes(3, probs, pars, C.byref(out)) == 0
    base = C.c_size_t()
    assert lib.isdc_batch_workspace_bytes(3, C.byref(base)) == 0
    plans = sum((_bytes(2, n, nu, fe, **kw)[1] + 255) // 256 * 256 for n, nu, fe, kw in
                [(63, 1.0, A.FE_ZERO, dict(precision=1)), (127, 0.5, A.FE_CUBIC, dict(precision=1, M=5)),
                 (31, 0.1, A.FE_ZERO, dict(precision=1))])
    assert out.value == base.value + plans
    h = C.c_void_p()
    fake = C.c_void_p(1 << 40)  # never dereferenced
    assert lib.isdc_batch_create(3, probs, pars, fake, out.value - 1, C.byref(h)) == A.E_WORKSPACE
    assert lib.isdc_batch_create(3, probs, pars, fake, out.value, C.byref(h)) == 0 and h.value
    us = (C.c_void_p * 3)(fake.value, None, fake.value)
    dts = (C.c_double * 3)(1e-3, 1e-3, 1e-3)
    assert lib.isdc_batch_step(h, us, dts, None, None, None) == A.E_INVAL          # d_u[1] NULL, all active
    bad = (C.c_double * 3)(1e-3, 1e-3, -1.0)
    act = (C.c_int32 * 3)(1, 0, 1)
    assert lib.isdc_batch_step(h, us, bad, act, None, None) == A.E_INVAL           # dt[2] <= 0
    assert b"dt[2]" in lib.isdc_last_error()
    lib.isdc_batch_destroy(h)
    # a slot batch (isdc_batch_open) has no fixed instances to step
    sb = C.c_void_p()
    assert lib.isdc_batch_open(3, 2, 1, 2, fake, base.value, C.byref(sb)) == 0
    assert lib.isdc_batch_step(sb, us, dts, act, None, None) == A.E_INVAL
    t, nl = C.c_double(), C.c_int32()
    assert lib.isdc_batch_time_sweeps(sb, 5, 0, None, C.byref(t), C.byref(nl)) == A.E_INVAL  # nothing running
    assert lib.isdc_batch_time_sweeps(sb, 5, 1, None, C.byref(t), C.byref(nl)) == A.E_INVAL  # graph on null stream
    assert lib.isdc_batch_time_sweeps(sb, 0, 0, fake, C.byref(t), C.byref(nl)) == A.E_INVAL
    lib.isdc_batch_destroy(sb)
    # instances must share dim, precision and L, and run the batch's solver
    mixed = (A.Params * 2)(make_params(precision=1), make_params(precision=0))
    two = (A.Problem * 2)(A.problem(2, 63, 1.0), A.problem(2, 63, 1.0))
    assert lib.isdc_batch_bytes(2, two, mixed, C.byref(out)) == A.E_INVAL
    # 2D weighted-Jacobi V(nu1, nu2) with nu1, nu2 <= 3 runs in a batch (beside red-black slots);
    # more steps, or Jacobi in 3D, do not
    jac = (A.Params * 2)(make_params(), make_params(smoother=A.SMOOTH_JACOBI, nu_pre=2, nu_post=3))
    assert lib.isdc_batch_bytes(2, two, jac, C.byref(out)) == 0
    jac4 = (A.Params * 2)(make_params(), make_params(smoother=A.SMOOTH_JACOBI, nu_pre=4, nu_post=4))
    assert lib.isdc_batch_bytes(2, two, jac4, C.byref(out)) == A.E_UNSUPPORTED
    cubes = (A.Problem * 2)(A.problem(3, 15, 1.0), A.problem(3, 15, 1.0))
    assert lib.isdc_batch_bytes(2, cubes, jac, C.byref(out)) == A.E_UNSUPPORTED
    dims = (A.Problem * 2)(A.problem(2, 63, 1.0), A.problem(3, 15, 1.0))
    assert lib.isdc_batch_bytes(2, dims, (A.Params * 2)(make_params(), make_params()), C.byref(out)) == A.E_INVAL
    assert lib.isdc_batch_bytes(0, two, mixed, C.byref(out)) == A.E_INVAL



def test_step_noalloc_rejects_before_device_work():
    lib = A.load()
    par = _params()
    st = A.Stats()
    # 1023^2 with M = 5 needs more than the static scratch
    big = A.problem(2, 1023, 1.0)
    p5 = _params(M=5)
    assert lib.isdc_step_noalloc(C.byref(big), C.byref(p5), C.c_void_p(1 << 40), 1e-3, None, C.byref(st)) == A.E_WORKSPACE
    assert b"static scratch" in lib.isdc_last_error()
    small = A.problem(2, 63, 1.0)
    assert lib.isdc_step_noalloc(C.byref(small), C.byref(par), None, 1e-3, None, C.byref(st)) == A.E_INVAL
    assert lib.isdc_step_noalloc(None, C.byref(par), C.c_void_p(1 << 40), 1e-3, None, C.byref(st)) == A.E_INVAL
