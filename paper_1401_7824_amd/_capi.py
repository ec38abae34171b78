"""ctypes declarations of the libisdc C ABI (include/isdc.h).

Argument marshalling only: every step of the method runs in the HIP library.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libisdc.so")

# status codes
OK, E_INVAL, E_WORKSPACE, E_HIP, E_NOT_CONVERGED, E_DIVERGED, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {OK: "ok", E_INVAL: "invalid", E_WORKSPACE: "workspace", E_HIP: "hip",
                E_NOT_CONVERGED: "not_converged", E_DIVERGED: "diverged", E_UNSUPPORTED: "unsupported"}
NODES_LOBATTO, NODES_RADAU_RIGHT, NODES_LEGENDRE = 0, 1, 2
FE_ZERO, FE_CUBIC, FE_BURGERS = 0, 1, 2
STENCIL_2ND, STENCIL_COMPACT4 = 0, 1
BC_DIRICHLET, BC_PERIODIC = 0, 1
SMOOTH_RBGS, SMOOTH_JACOBI = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
GUESS_PREV_SWEEP, GUESS_ZERO, GUESS_PREV_NODE = 0, 1, 2
OP_SMOOTH, OP_RESTRICT, OP_PROLONG, OP_COARSE, OP_RESIDUAL_NORM, OP_EXPLICIT = 0, 1, 2, 3, 4, 5
KERNEL_SMOOTH_RESTRICT, KERNEL_PROLONG_SMOOTH, KERNEL_SMOOTH, KERNEL_TAIL, KERNEL_QUAD, KERNEL_EXPLICIT = 0, 1, 2, 3, 4, 5
KERNEL_PROLONG_UPDATE, KERNEL_RESTRICT, KERNEL_RHS = 6, 7, 8
SLOT_FREE, SLOT_RUNNING, SLOT_FINISHED = 0, 1, 2
MAX_M = 9
HIST = 128


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("nu", C.c_double), ("fe_kind", C.c_int32),
                ("stencil", C.c_int32), ("bc", C.c_int32)]


def problem(dim, n, nu, fe_kind=FE_ZERO, stencil=STENCIL_2ND, bc=BC_DIRICHLET) -> Problem:
    """isdc_problem of a grid with n points on each of the dim axes (n[a] = 1 beyond)."""
    axes = (C.c_int32 * 3)(*[n if a < dim else 1 for a in range(3)])
    return Problem(dim=dim, n=axes, nu=nu, fe_kind=fe_kind, stencil=stencil, bc=bc)


class Params(C.Structure):
    _fields_ = [("node_kind", C.c_int32), ("M", C.c_int32), ("vcycles", C.c_int32),
                ("inner_tol", C.c_double), ("early_exit", C.c_int32), ("sdc_tol", C.c_double),
                ("max_sweeps", C.c_int32), ("smoother", C.c_int32), ("nu_pre", C.c_int32),
                ("nu_post", C.c_int32), ("precision", C.c_int32), ("guess", C.c_int32), ("levels", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("hist_len", C.c_int32), ("vcycles", C.c_int64),
                ("residual", C.c_double), ("residual_hist", C.c_double * HIST), ("coarse_vcycles", C.c_int64)]


# (name, restype, argtypes) for every function declared in include/isdc.h
_VP, _DP, _SZP = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_size_t)
SIGNATURES = [
    ("isdc_version", C.c_int, []),
    ("isdc_abi_sizes", C.c_int, [_SZP, _SZP, _SZP]),
    ("isdc_last_error", C.c_char_p, []),
    ("isdc_default_params", C.c_int, [C.POINTER(Params)]),
    ("isdc_tables", C.c_int, [C.c_int32, C.c_int32, _DP, _DP, _DP]),
    ("isdc_end_weights", C.c_int, [C.c_int32, C.c_int32, _DP]),
    ("isdc_workspace_bytes", C.c_int, [C.POINTER(Problem), C.POINTER(Params), _SZP]),
    ("isdc_create", C.c_int, [C.POINTER(Problem), C.POINTER(Params), _VP, C.c_size_t, C.POINTER(_VP)]),
    ("isdc_destroy", None, [_VP]),
    ("isdc_step", C.c_int, [_VP, _VP, C.c_double, _VP, C.POINTER(Stats)]),
    ("isdc_step_noalloc", C.c_int, [C.POINTER(Problem), C.POINTER(Params), _VP, C.c_double, _VP, C.POINTER(Stats)]),
    ("isdc_begin", C.c_int, [_VP, _VP, C.c_double, _VP]),
    ("isdc_sweep", C.c_int, [_VP, _VP, _DP]),
    ("isdc_end", C.c_int, [_VP, _VP, _VP]),
    ("isdc_node_values", C.c_int, [_VP, C.c_int32, _VP, _VP]),
    ("isdc_get_stats", C.c_int, [_VP, C.POINTER(Stats)]),
    ("isdc_vcycle", C.c_int, [_VP, C.c_double, C.c_int32, _VP, _VP, C.c_int32, _VP, _DP]),
    ("isdc_mg_op", C.c_int, [_VP, C.c_int32, C.c_int32, C.c_double, C.c_int32, _VP, _VP, _VP, _VP, _DP]),
    ("isdc_time_kernel", C.c_int, [_VP, C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_int32, _VP, _DP, _DP]),
    ("isdc_probe_arm", C.c_int, [_VP, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    ("isdc_probe_read", C.c_int, [_VP, C.POINTER(C.c_int64), _DP, _DP]),
    ("isdc_autotune", C.c_int, [_VP, C.c_int32, _VP, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    ("isdc_set_tile_shapes", C.c_int, [_VP, C.POINTER(C.c_int32), C.c_int32]),
    ("isdc_get_tile_shapes", C.c_int, [_VP, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
    ("isdc_batch_bytes", C.c_int, [C.c_int32, C.POINTER(Problem), C.POINTER(Params), _SZP]),
    ("isdc_batch_create", C.c_int, [C.c_int32, C.POINTER(Problem), C.POINTER(Params), _VP, C.c_size_t,
                                    C.POINTER(_VP)]),
    ("isdc_batch_step", C.c_int, [_VP, C.POINTER(_VP), _DP, C.POINTER(C.c_int32), _VP, C.POINTER(Stats)]),
    ("isdc_batch_workspace_bytes", C.c_int, [C.c_int32, _SZP]),
    ("isdc_batch_open", C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _VP, C.c_size_t, C.POINTER(_VP)]),
    ("isdc_batch_destroy", None, [_VP]),
    ("isdc_batch_set", C.c_int, [_VP, C.c_int32, C.POINTER(Problem), C.POINTER(Params), _VP, C.c_size_t, _VP,
                                 C.c_double, C.c_int32]),
    ("isdc_batch_advance", C.c_int, [_VP, _VP, C.POINTER(C.c_int32)]),
    ("isdc_batch_time_sweeps", C.c_int, [_VP, C.c_int32, C.c_int32, _VP, _DP, C.POINTER(C.c_int32)]),
    ("isdc_batch_slot_info", C.c_int, [_VP, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(Stats)]),
    ("isdc_batch_release", C.c_int, [_VP, C.c_int32]),
]

_lib = None


class ISDCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libisdc.so (cached).  Raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1401_7824_amd.build`")
    # torch brings its own HIP runtime; load it first so that the library binds
    # to that one instead of starting a second runtime beside it
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    sizes = [C.c_size_t() for _ in range(3)]
    lib.isdc_abi_sizes(*[C.byref(s) for s in sizes])
    mine = (C.sizeof(Problem), C.sizeof(Params), C.sizeof(Stats))
    if tuple(s.value for s in sizes) != mine:
        raise RuntimeError(f"struct layout mismatch: library {[s.value for s in sizes]}, binding {mine}")
    _lib = lib
    return lib


def check(rc, allow=()):
    """Raise ISDCError unless rc is OK or listed in `allow`; returns rc."""
    if rc != OK and rc not in allow:
        raise ISDCError(rc, load().isdc_last_error().decode())
    return rc
