"""MI355X (gfx950) implementation of inexact spectral deferred corrections.

The HIP library libisdc.so (C ABI in include/isdc.h) does all the work; this
package is a thin binding over it.  The library is loaded on first use and
its absence is an error.
"""
from ._capi import (  # noqa: F401
    ISDCError, NODES_LOBATTO, NODES_RADAU_RIGHT, NODES_LEGENDRE, FE_ZERO, FE_CUBIC, FE_BURGERS, STENCIL_2ND, STENCIL_COMPACT4,
    BC_DIRICHLET, BC_PERIODIC,
    SMOOTH_RBGS, SMOOTH_JACOBI, PREC_FP64, PREC_MIXED, GUESS_PREV_SWEEP, GUESS_ZERO, GUESS_PREV_NODE,
    OP_SMOOTH, OP_RESTRICT, OP_PROLONG, OP_COARSE, OP_RESIDUAL_NORM, OP_EXPLICIT, load,
    KERNEL_SMOOTH_RESTRICT, KERNEL_PROLONG_SMOOTH, KERNEL_SMOOTH, KERNEL_TAIL, KERNEL_QUAD, KERNEL_EXPLICIT,
    KERNEL_PROLONG_UPDATE, KERNEL_RESTRICT, KERNEL_RHS,
    SLOT_FREE, SLOT_RUNNING, SLOT_FINISHED,
)


def __getattr__(name):
    # the torch-based binding is imported lazily so that the C-ABI checks and the
    # input generators work without touching a GPU
    if name in ("Plan", "Batch", "FixedBatch", "StepStats", "tables", "end_weights", "make_params", "make_problem",
                "workspace_bytes", "step_noalloc"):
        from . import isdc
        return getattr(isdc, name)
    raise AttributeError(name)
