"""Plain FP64 CPU oracle for inexact spectral deferred corrections (ISDC).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never calls into it and shares no code with it: no kernels, headers, helpers,
tables or constant generators.  It is written from the paper (Speck,
Ruprecht, Minion, Emmett, Krause, "Inexact spectral deferred corrections")
and from the textbook definitions it relies on, in numpy (plus scipy.fft and
mpmath), slow and direct on purpose.

Module map (each function cites the passage it follows):

* ``collocation`` -- collocation nodes on [0, 1] (Sec. 1, Sec. 2 around
  eq. (2)), the cumulative quadrature matrix Q and the node-to-node matrix S of
  eq. (2), and the direct collocation solution (Sec. 1: the large coupled
  system that SDC approximates).
* ``operators`` -- the second-order finite-difference Laplacian with
  homogeneous Dirichlet boundary, the split f = f^I + f^E of eq. (4), and the
  exact shifted-Laplacian solve by sine transform.
* ``multigrid`` -- the geometric multigrid V-cycle used as the inner solver
  (Sec. 3), in float64 or float32.
* ``compact`` -- the fourth-order compact Laplacian A_h and its weighting
  matrix W (Sec. 3, eq. (5)), their exact solves by sine transform and the
  weighted-Jacobi V-cycle for W - c A_h.
* ``periodic`` -- periodic grids on [-1, 1)^d, the periodic compact stencil,
  its Fourier solves and multigrid, and the WENO5 advection of viscous
  Burgers (Sec. 4.1).
* ``mlsdc`` -- two-level MLSDC with ISDC sweeps: a spatially coarsened
  level tied to the fine one by an FAS term (Sec. 5).
* ``sdc`` -- the semi-implicit SDC sweep of eq. (4) (and of eq. (5) for the
  compact stencil) with exact, classical (solve to tolerance) and inexact
  (L V-cycles) inner solves, the SDC residual of Sec. 3, and the time step.

Parity pins for every function live in ``tests/test_oracle_*.py``.  Nothing
here is "parity unpinned".
"""

from .collocation import (  # noqa: F401
    NODES_LOBATTO,
    NODES_RADAU_RIGHT,
    NODES_LEGENDRE,
    nodes,
    end_weights,
    qmatrix,
    smatrix,
    collocation_heat_modal,
    collocation_dense,
    stability_function,
)
from .operators import (  # noqa: F401
    FE_ZERO,
    FE_CUBIC,
    laplacian,
    f_explicit,
    f_implicit,
    apply_shifted,
    solve_shifted_exact,
    laplacian_eigenvalues,
)
from .multigrid import (  # noqa: F401
    SMOOTH_RBGS,
    SMOOTH_JACOBI,
    vcycle,
    smooth,
    restrict_fw,
    prolong_linear,
    level_sizes,
)
from .compact import (  # noqa: F401
    laplacian_compact,
    weight,
    compact_eigenvalues,
    solve_weight_exact,
    solve_compact_shifted_exact,
    apply_compact_shifted,
    vcycle_compact,
)
from .periodic import (  # noqa: F401
    grid_p,
    laplacian_compact_p,
    weight_p,
    burgers_advection,
    vcycle_compact_p,
)
from .sdc import (  # noqa: F401
    STENCIL_2ND,
    STENCIL_COMPACT4,
    BC_DIRICHLET,
    BC_PERIODIC,
    FE_BURGERS,
    SDCConfig,
    SDCStats,
    sdc_step,
    sdc_residual,
    SDCState,
    sdc_begin,
    sdc_sweep,
    NotConverged,
    Diverged,
)
