"""GPU parity of the multigrid kernels against the oracle (through the C ABI).

Sizes span several 256-wide row tiles with a ragged tail and, for the
V-cycle, both the multi-workgroup levels and the single-workgroup coarse tail.
FP64 results must match the oracle's float64 arithmetic to rounding; FP32
kernels match the oracle's float32 arithmetic to float32 rounding.
"""

import numpy as np
import pytest
import torch

import oracle as O
from gpu_helpers import announce, dev, host, rel_l2, require_gpu, random_field

pytestmark = pytest.mark.gpu

RBGS, JAC = O.SMOOTH_RBGS, O.SMOOTH_JACOBI
# level-0 sizes per dimension: 1D beyond the 2047-point tail, 2D / 3D with
# multi-workgroup levels above the tail
SIZES = {1: 4095, 2: 255, 3: 63}
TOL = {torch.float64: 1e-13, torch.float32: 2e-6}


def _plan(d, n, smoother, nu_pre=None, nu_post=None):
    from paper_1401_7824_amd import Plan
    if nu_pre is None:
        nu_pre, nu_post = (1, 1) if smoother == RBGS else (2, 2)
    return Plan(d, n, 1.0, smoother=smoother, nu_pre=nu_pre, nu_post=nu_post)


def _np_dtype(tdt):
    return np.float64 if tdt == torch.float64 else np.float32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("smoother", [RBGS, JAC])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_smoother_parity(d, smoother, dtype):
    n = SIZES[d]
    announce("smooth", d, n, smoother, dtype)
    p = _plan(d, n, smoother)
    h = 1.0 / (n + 1)
    c = 37.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n,) * d, 1).astype(nd)
    u = random_field((n,) * d, 2).astype(nd)
    out = torch.empty((n,) * d, dtype=dtype, device="cuda")
    p.mg_op(O_op("SMOOTH"), 0, c, a=dev(rhs, dtype), b=dev(u, dtype), out=out)
    ref = O.smooth(u, rhs, c, h, smoother)
    assert ref.dtype == nd
    assert rel_l2(host(out), ref) < TOL[dtype]


def O_op(name):
    import paper_1401_7824_amd as P
    return getattr(P, "OP_" + name)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_restrict_and_prolong_parity(d, dtype):
    n = SIZES[d]
    announce("transfer", d, n, dtype)
    p = _plan(d, n, RBGS)
    h = 1.0 / (n + 1)
    c = 11.0 * h * h
    nd = _np_dtype(dtype)
    nc = (n - 1) // 2
    rhs = random_field((n,) * d, 3).astype(nd)
    u = random_field((n,) * d, 4).astype(nd)
    rc = torch.empty((nc,) * d, dtype=dtype, device="cuda")
    p.mg_op(O_op("RESTRICT"), 0, c, a=dev(rhs, dtype), b=dev(u, dtype), out=rc)
    ref = O.restrict_fw(rhs - O.apply_shifted(u, c, h))
    assert rel_l2(host(rc), ref) < TOL[dtype]
    ec = random_field((nc,) * d, 5).astype(nd)
    ud = dev(u, dtype)
    p.mg_op(O_op("PROLONG"), 0, c, a=dev(ec, dtype), out=ud)
    assert rel_l2(host(ud), u + O.prolong_linear(ec)) < TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("smoother", [RBGS, JAC])
@pytest.mark.parametrize("d,n", [(1, 2047), (1, 127), (2, 63), (2, 7), (3, 15), (3, 3), (2, 1)])
def test_coarse_tail_parity(d, n, smoother, dtype):
    announce("tail", d, n, smoother, dtype)
    p = _plan(d, n, smoother)
    h = 1.0 / (n + 1)
    c = 25.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n,) * d, 6).astype(nd)
    out = torch.empty((n,) * d, dtype=dtype, device="cuda")
    p.mg_op(O_op("COARSE"), 0, c, a=dev(rhs, dtype), out=out)
    nu1 = 1 if smoother == RBGS else 2
    ref = O.vcycle(np.zeros_like(rhs), rhs, c, h, smoother, nu1, nu1)
    assert rel_l2(host(out), ref) < TOL[dtype] * 5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("smoother", [RBGS, JAC])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_vcycle_parity(d, smoother, dtype):
    n = SIZES[d]
    announce("vcycle", d, n, smoother, dtype)
    p = _plan(d, n, smoother)
    h = 1.0 / (n + 1)
    c = 64.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n,) * d, 7).astype(nd)
    u0 = random_field((n,) * d, 8).astype(nd)
    u = dev(u0, dtype)
    res = p.vcycle(c, dev(rhs, dtype), u, ncycles=2, want_residual=True)
    nu1 = 1 if smoother == RBGS else 2
    ref = u0
    for _ in range(2):
        ref = O.vcycle(ref, rhs, c, h, smoother, nu1, nu1)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert rel_l2(host(u), ref) < tol
    ref_res = float(np.max(np.abs(rhs.astype(np.float64) - O.apply_shifted(ref.astype(np.float64), c, h))))
    assert abs(res - ref_res) <= 1e-3 * ref_res + (1e-12 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("d,n,stiff", [(1, 511, 80.0), (2, 127, 80.0), (3, 31, 40.0)])
def test_vcycle_contraction_matches_oracle(d, n, stiff):
    announce("contraction", d, n)
    p = _plan(d, n, RBGS)
    h = 1.0 / (n + 1)
    c = stiff * h * h
    e0 = random_field((n,) * d, 9)
    zero = torch.zeros((n,) * d, dtype=torch.float64, device="cuda")
    e = dev(e0)
    est_gpu = 0.0
    for _ in range(40):
        before = torch.linalg.vector_norm(e).item()
        p.vcycle(c, zero, e, ncycles=1)
        after = torch.linalg.vector_norm(e).item()
        est_gpu = after / before
        e /= after
    eo = e0.copy()
    est_cpu = 0.0
    z = np.zeros_like(eo)
    for _ in range(40):
        e2 = O.vcycle(eo, z, c, h)
        est_cpu = np.linalg.norm(e2) / np.linalg.norm(eo)
        eo = e2 / np.linalg.norm(e2)
    assert 0.0 < est_cpu < 0.4
    assert abs(est_gpu - est_cpu) <= 1e-6 * est_cpu


def test_residual_norm_parity():
    announce("resnorm")
    n = 255
    p = _plan(2, n, RBGS)
    h = 1.0 / (n + 1)
    c = 3.0 * h * h
    rhs = random_field((n, n), 10)
    u = random_field((n, n), 11)
    r = p.mg_op(O_op("RESIDUAL_NORM"), 0, c, a=dev(rhs), b=dev(u))
    ref = float(np.max(np.abs(rhs - O.apply_shifted(u, c, h))))
    assert abs(r - ref) <= 1e-13 * ref


def test_time_kernel_reports_durations_and_bytes():
    announce("time_kernel")
    import paper_1401_7824_amd as P
    n = 255
    p = _plan(2, n, RBGS)
    h = 1.0 / (n + 1)
    c = 10 * h * h
    N, Nc = n * n, 127 * 127
    for k, expect in [(P.KERNEL_SMOOTH_RESTRICT, (3 * N + Nc) * 8), (P.KERNEL_PROLONG_SMOOTH, (3 * N + Nc) * 8),
                      (P.KERNEL_SMOOTH, 3 * N * 8), (P.KERNEL_TAIL, 2 * 63 * 63 * 8)]:
        us, b = p.time_kernel(k, 0, c, 0, reps=5)
        assert 0.0 < us < 1e4
        assert b == expect
    with pytest.raises(Exception):
        p.time_kernel(P.KERNEL_QUAD, 0, c, 0, reps=2)  # no step in progress
    with pytest.raises(Exception):
        p.time_kernel(P.KERNEL_SMOOTH, 3, c, 0, reps=2)  # level 3 is the coarse tail


# ---- tile shapes: every shape computes the same V-cycle ----

SHAPE_SIZES = {1: 8191, 2: 511, 3: 63}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_vcycle_parity_every_tile_shape(d, shape, dtype):
    n = SHAPE_SIZES[d]
    announce("vcycle shape", d, n, shape, dtype)
    p = _plan(d, n, RBGS, nu_pre=2, nu_post=2)
    nl = len(p.tile_shapes)
    assert nl >= 2
    p.tile_shapes = [shape] * nl
    assert p.tile_shapes == [shape] * nl
    h = 1.0 / (n + 1)
    c = 64.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n,) * d, 17).astype(nd)
    u0 = random_field((n,) * d, 18).astype(nd)
    u = dev(u0, dtype)
    p.vcycle(c, dev(rhs, dtype), u, ncycles=2)
    ref = u0
    for _ in range(2):
        ref = O.vcycle(ref, rhs, c, h, RBGS, 2, 2)
    assert rel_l2(host(u), ref) < (1e-12 if dtype == torch.float64 else 2e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vcycle_parity_every_march_depth(dtype):
    # 3D levels of 127^3 and up are z-marched; the shape picks the column
    # depth (2, 4 or 8 planes at 127^3, the 63^3 level below uses tiles)
    n, d = 127, 3
    h = 1.0 / (n + 1)
    c = 64.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n,) * d, 27).astype(nd)
    u0 = random_field((n,) * d, 28).astype(nd)
    ref = u0
    for _ in range(2):
        ref = O.vcycle(ref, rhs, c, h, RBGS, 2, 2)
    for shape in (0, 1, 2):
        announce("vcycle march depth", n, shape, dtype)
        p = _plan(d, n, RBGS, nu_pre=2, nu_post=2)
        p.tile_shapes = [shape] * len(p.tile_shapes)
        u = dev(u0, dtype)
        p.vcycle(c, dev(rhs, dtype), u, ncycles=2)
        assert rel_l2(host(u), ref) < (1e-12 if dtype == torch.float64 else 2e-5), shape


def test_vcycle_v11_zero_start_marched_level_parity():
    # V(1,1) on 255^3: the 127^3 level starts every cycle from zero, so its
    # first red-black step runs fused with the residual's restriction
    # (k_march_zrestrict); 255^3 and 127^3 are both z-marched
    n, d = 255, 3
    h = 1.0 / (n + 1)
    c = 64.0 * h * h
    rhs = random_field((n,) * d, 37)
    u0 = random_field((n,) * d, 38)
    for dtype in (torch.float64, torch.float32):
        nd = _np_dtype(dtype)
        ref = u0.astype(nd)
        for _ in range(2):
            ref = O.vcycle(ref, rhs.astype(nd), c, h, RBGS, 1, 1)
        announce("vcycle V(1,1) 255^3", dtype)
        p = _plan(d, n, RBGS, nu_pre=1, nu_post=1)
        u = dev(u0, dtype)
        p.vcycle(c, dev(rhs, dtype), u, ncycles=2)
        assert rel_l2(host(u), ref) < (1e-12 if dtype == torch.float64 else 2e-5), dtype


def test_autotune_picks_valid_shapes_and_keeps_results(tmp_path, monkeypatch):
    from paper_1401_7824_amd import ISDCError
    announce("autotune")
    monkeypatch.setenv("ISDC_TUNE_CACHE", str(tmp_path / "tiles.json"))
    n = 511
    p = _plan(2, n, RBGS)
    shapes = p.autotune(reps=5)
    assert len(shapes) == len(p.tile_shapes) and all(0 <= s < 3 for s in shapes)
    assert p.tile_shapes == shapes
    q = _plan(2, n, RBGS)
    assert q.autotune(reps=5) == shapes  # from the cache
    h = 1.0 / (n + 1)
    c = 64.0 * h * h
    rhs = random_field((n, n), 19)
    u = dev(np.zeros((n, n)))
    p.vcycle(c, dev(rhs), u, ncycles=2)
    ref = O.vcycle(O.vcycle(np.zeros((n, n)), rhs, c, h, RBGS, 1, 1), rhs, c, h, RBGS, 1, 1)
    assert rel_l2(host(u), ref) < 1e-12
    with pytest.raises(ISDCError):
        p.tile_shapes = [3] * len(shapes)
    with pytest.raises(ISDCError):
        p.tile_shapes = [0] * (len(shapes) + 1)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("nu1,nu2", [(1, 1), (2, 2), (3, 3), (4, 5), (0, 2), (2, 0)])
def test_jacobi_2d_fused_vcycle_parity(nu1, nu2, dtype):
    # 2D weighted-Jacobi cycles run fused row-tile launches (up to three steps
    # with the restriction, the prolongation with up to three steps); every
    # split of the smoothing steps over the launches gives the oracle's cycle
    n = 255
    announce("jacobi fused vcycle", nu1, nu2, dtype)
    p = _plan(2, n, JAC, nu1, nu2)
    h = 1.0 / (n + 1)
    c = 80.0 * h * h
    nd = _np_dtype(dtype)
    rhs = random_field((n, n), 17).astype(nd)
    u0 = random_field((n, n), 18).astype(nd)
    u = dev(u0, dtype)
    p.vcycle(c, dev(rhs, dtype), u, ncycles=2)
    ref = u0
    for _ in range(2):
        ref = O.vcycle(ref, rhs, c, h, JAC, nu1, nu2)
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert rel_l2(host(u), ref) < tol
