"""Shared helpers of the GPU parity tests (imported only by tests marked gpu)."""

import sys

import numpy as np
import torch


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device (run them with -m gpu on an MI355X)")


def announce(*parts):
    """Name the case on stdout before any device work, so a failure is traceable."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def random_field(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)
