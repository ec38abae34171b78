"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only builds inputs; it holds none of the method's arithmetic.
Every initial value is a sum of discrete sine modes prod_i sin(a_i pi x_i) on
the interior points x_i = (i + 1) h, h = 1 / (n + 1) of [0, 1]^d, which
satisfy the homogeneous Dirichlet boundary condition:

* the wave vectors a are drawn uniformly without replacement from
  {1..max_wave}^d with numpy's default_rng(seed);
* each amplitude is standard normal divided by |a|^2 (a smooth field, as for
  the paper's smooth initial data in Sec. 4.1).

Periodic inputs live on the n points x_i = -1 + i h, h = 2 / n of [-1, 1)
per axis: the Gaussian exp(-|x|^2 / sigma^2) of the Burgers runs (Sec. 4.1,
sigma = 0.1), and seeded smooth fields sum_k amp_k cos(pi a.x + phi_k) with
integer wave vectors a (period 2 in every coordinate).

The workload table mirrors the benchmark configurations (sizes, nodes, time
step, precision); no public dataset is involved.
"""
from __future__ import annotations

import numpy as np

NODES_LOBATTO, NODES_RADAU_RIGHT, NODES_LEGENDRE = 0, 1, 2
FE_ZERO, FE_CUBIC, FE_BURGERS = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1


def draw_modes(d: int, n_modes: int, seed: int, max_wave: int = 8):
    """List of (amplitude, wave vector) pairs; see the module docstring."""
    rng = np.random.default_rng(seed)
    grid = np.stack(np.meshgrid(*[np.arange(1, max_wave + 1)] * d, indexing="ij"), -1).reshape(-1, d)
    pick = rng.choice(len(grid), size=n_modes, replace=False)
    modes = []
    for idx in pick:
        a = tuple(int(v) for v in grid[idx])
        amp = rng.standard_normal() / float(sum(v * v for v in a))
        modes.append((amp, a))
    return modes


def sine_field(n: int, d: int, modes) -> np.ndarray:
    """Evaluate sum_k amp_k prod_i sin(a_ki pi x_i) on the n^d interior grid (float64)."""
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    u = np.zeros((n,) * d)
    for amp, a in modes:
        term = np.asarray(amp, dtype=np.float64)
        for ax in range(d):
            shape = [1] * d
            shape[ax] = n
            term = term * np.sin(a[ax] * np.pi * x).reshape(shape)
        u += term
    return u


def sine_field_device(n: int, d: int, modes, device="cuda"):
    """sine_field built on a torch device: the 1D sine vectors are evaluated
    on the host in float64 and their products formed on the device in the
    same order as sine_field, so the result equals sine_field bit for bit."""
    import torch
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    u = torch.zeros((n,) * d, dtype=torch.float64, device=device)
    for amp, a in modes:
        term = torch.tensor(float(amp), dtype=torch.float64, device=device)
        for ax in range(d):
            shape = [1] * d
            shape[ax] = n
            term = term * torch.from_numpy(np.sin(a[ax] * np.pi * x)).to(device).reshape(shape)
        u += term
    return u


def sine_field_at(n: int, modes, points: np.ndarray) -> np.ndarray:
    """The same field at integer grid points (rows of `points`, one column per axis)."""
    h = 1.0 / (n + 1)
    xs = (np.asarray(points) + 1) * h
    out = np.zeros(len(xs))
    for amp, a in modes:
        term = np.full(len(xs), amp)
        for ax, ai in enumerate(a):
            term *= np.sin(ai * np.pi * xs[:, ax])
        out += term
    return out


def periodic_axis(n: int) -> np.ndarray:
    """The n grid coordinates of [-1, 1) (spacing 2 / n)."""
    return -1.0 + (2.0 / n) * np.arange(n)


def gaussian_periodic(n: int, sigma: float = 0.1, d: int = 2) -> np.ndarray:
    """exp(-|x|^2 / sigma^2) on the periodic n^d grid of [-1, 1)^d (float64)."""
    x = periodic_axis(n)
    r2 = np.zeros((n,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = n
        r2 = r2 + (x ** 2).reshape(shape)
    return np.exp(-r2 / sigma ** 2)


def periodic_field(n: int, seed: int, n_modes: int = 8, max_wave: int = 6, d: int = 2) -> np.ndarray:
    """Seeded smooth periodic field: sum of n_modes cos(pi a.x + phi), a in
    {-max_wave..max_wave}^d, amplitude N(0,1) / (1 + |a|^2), phase U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    x = periodic_axis(n)
    grids = np.meshgrid(*([x] * d), indexing="ij")
    out = np.zeros((n,) * d)
    for _ in range(n_modes):
        a = rng.integers(-max_wave, max_wave + 1, size=d)
        amp = rng.standard_normal() / (1.0 + float(np.dot(a, a)))
        phi = rng.uniform(0.0, 2.0 * np.pi)
        out += amp * np.cos(np.pi * sum(ai * g for ai, g in zip(a, grids)) + phi)
    return out


# The five workloads of the benchmark: sizes, nodes, step and precision.
WORKLOADS = {
    "heat1d": dict(dim=1, n=127, nu=1.0, fe_kind=FE_ZERO, node_kind=NODES_LOBATTO, M=3, dt=0.01, steps=1,
                   precision=PREC_FP64, sdc_tol=1e-10, modes=[(1.0, (1,)), (0.5, (3,))]),
    # weighted-Jacobi V(3,3): the fewest V-cycles and the least time per step of the
    # smoothers measured on this problem (bench.py --workload compare)
    "rd2d": dict(dim=2, n=1023, nu=0.1, fe_kind=FE_CUBIC, node_kind=NODES_LOBATTO, M=5, dt=1e-3, steps=10,
                 precision=PREC_FP64, sdc_tol=1e-10, n_modes=16, seed=2, smoother=1, nu_pre=3, nu_post=3),
    # all-float64; bench.py runs the float32-V-cycle variant beside it
    "heat3d": dict(dim=3, n=255, nu=1.0, fe_kind=FE_ZERO, node_kind=NODES_RADAU_RIGHT, M=3, dt=1e-3, steps=1,
                   precision=PREC_FP64, sdc_tol=1e-10, n_modes=32, seed=3),
    # the rd2d problem with the fourth-order compact stencil and weighting matrix W
    # (weighted-Jacobi V(2,2) cycles for W - dt_m nu A_h)
    "rd2d_compact": dict(dim=2, n=1023, nu=0.1, fe_kind=FE_CUBIC, node_kind=NODES_LOBATTO, M=5, dt=1e-3, steps=10,
                         precision=PREC_FP64, sdc_tol=1e-10, n_modes=16, seed=2, stencil=1, smoother=1,
                         nu_pre=2, nu_post=2),
    # the rd2d problem with two-level MLSDC (ISDC sweeps on 1023^2 and 511^2, FAS, cubic interpolation)
    "rd2d_mlsdc": dict(dim=2, n=1023, nu=0.1, fe_kind=FE_CUBIC, node_kind=NODES_LOBATTO, M=5, dt=1e-3, steps=10,
                       precision=PREC_FP64, sdc_tol=1e-10, n_modes=16, seed=2, levels=2),
    # 2D viscous Burgers of Sec. 4.1 on [-1, 1)^2, periodic, 128^2 points (h = 1/64),
    # Gaussian sigma = 0.1, nu = 1 (diffusive CFL 4.1), WENO5 advection, compact stencil
    "burgers2d": dict(dim=2, n=128, nu=1.0, fe_kind=FE_BURGERS, node_kind=NODES_LOBATTO, M=5, dt=1e-3, steps=10,
                      precision=PREC_FP64, sdc_tol=1e-10, stencil=1, bc=1, smoother=1, nu_pre=3, nu_post=3,
                      gaussian_sigma=0.1),
}


def workload_modes(cfg: dict):
    if "modes" in cfg:
        return list(cfg["modes"])
    return draw_modes(cfg["dim"], cfg["n_modes"], cfg["seed"])


def workload_u0(cfg: dict, n: int | None = None) -> np.ndarray:
    """Initial value of a workload (optionally on a smaller grid of the same modes)."""
    n = cfg["n"] if n is None else n
    if "gaussian_sigma" in cfg:
        return gaussian_periodic(n, cfg["gaussian_sigma"], cfg["dim"])
    return sine_field(n, cfg["dim"], workload_modes(cfg))


def batch_instances(count: int = 256, seed0: int = 4000, param_seed: int = 4):
    """Parameters of the batched workload: 2D reaction-diffusion instances with
    side 2^k - 1, k uniform in {6..9}, nu ~ U[0.01, 1], dt ~ U[1e-4, 1e-2],
    M uniform in {3, 5} (Gauss-Lobatto), 16 modes, instance i seeded 4000 + i."""
    rng = np.random.default_rng(param_seed)
    out = []
    for i in range(count):
        k = int(rng.integers(6, 10))
        out.append(dict(dim=2, n=2 ** k - 1, nu=float(rng.uniform(0.01, 1.0)), fe_kind=FE_CUBIC,
                        node_kind=NODES_LOBATTO, M=int(rng.choice([3, 5])), dt=float(rng.uniform(1e-4, 1e-2)),
                        precision=PREC_MIXED, sdc_tol=1e-8, n_modes=16, seed=seed0 + i))
    return out
