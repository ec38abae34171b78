/*
 * isdc.h -- C ABI of libisdc, an MI355X (gfx950) implementation of inexact
 * spectral deferred corrections (ISDC; Speck, Ruprecht, Minion, Emmett and
 * Krause, "Inexact spectral deferred corrections").
 *
 * Problem (Sec. 2, eq. (1)):  u' = f(u) = f^I(u) + f^E(u) on [0,1]^d,
 *   f^I(u) = nu * L_h u  -- the (2d+1)-point second-order Laplacian on the
 *                           n^d interior points x_i = (i+1) h, h = 1/(n+1),
 *                           homogeneous Dirichlet boundary (Sec. 3: the
 *                           linearly implicit case f^I = A u);
 *   f^E(u) = 0 (heat equation, Sec. 4.1) or u - u^3 (reaction-diffusion).
 * One time step of length dt runs semi-implicit SDC sweeps (eq. (4)) over M
 * collocation nodes; every implicit Euler system (I - dt_m nu L_h) u = rhs is
 * solved only approximately by L geometric-multigrid V-cycles warm-started
 * from the previous sweep (Sec. 3, Sec. 4.3), and sweeps continue until the
 * max-norm SDC residual (Sec. 3) is below a tolerance.
 *
 * With the fourth-order compact stencil (isdc_problem.stencil, 2D only) f^I
 * is nu W^{-1} A_h with the 9-point A_h = L_h + (h^2/6) D_x D_y and the
 * weighting matrix W = I + (h^2/12) L_h; the sweep is eq. (5), whose systems
 * (W - dt_m nu A_h) u = rhs are solved by weighted-Jacobi V-cycles, and the
 * SDC residual inverts W once per node (Sec. 3).
 *
 * Conventions shared by every entry point:
 *  - Grid arrays are dense, row-major n^d arrays of the interior points with
 *    the x index fastest (numpy C order of shape (n,)*d).  No ghost points.
 *  - Device pointers (prefix d_) point to memory on the current HIP device,
 *    allocated and owned by the caller; the library never allocates or frees
 *    device memory.  Host pointers (prefix h_) are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is enqueued on it; entry points that must read a result back
 *    say so and synchronise that stream.
 *  - Every function returns an isdc_status (0 = success).  On failure a
 *    message is available from isdc_last_error() (per thread).  Arguments are
 *    validated before any device work is enqueued; an invalid argument leaves
 *    device memory untouched.  No C++ exception crosses this interface.
 *  - A plan is not thread safe: calls on one plan must not overlap.
 *  - Tracing: with the environment variable ISDC_TRACE set ("1" or "stderr":
 *    standard error; any other non-empty value except "0": a file path the
 *    lines are appended to; read once per process) every sweep of
 *    isdc_step and every batch sweep writes one line with the host time
 *    after its residual read-back ("isdc_trace plan=... sweep=... t_us=...
 *    residual=... vcycles=..." / "isdc_trace batch=... running=... t_us=...").
 */
#ifndef ISDC_H
#define ISDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ISDC_OK = 0,
    ISDC_E_INVAL = -1,          /* invalid argument (nothing was enqueued)              */
    ISDC_E_WORKSPACE = -2,      /* workspace too small or misaligned                    */
    ISDC_E_HIP = -3,            /* a HIP runtime call failed                            */
    ISDC_E_NOT_CONVERGED = -4,  /* max_sweeps reached; the last iterate was written     */
    ISDC_E_DIVERGED = -5,       /* non-finite SDC residual; the last iterate was written */
    ISDC_E_UNSUPPORTED = -6     /* valid request the library does not implement         */
} isdc_status;

/* Collocation node families (Sec. 1; Sec. 2 after eq. (2)).  Gauss-Lobatto
 * and right Gauss-Radau end on tau_M = 1, so a step's result is u_M;
 * Gauss-Legendre nodes are all interior and a step's result is the end-point
 * quadrature u_0 + dt sum_j b_j f(u_j) (isdc_end_weights; compact stencil:
 * u_0 + W^{-1}(dt sum_j b_j f~_j)). */
enum { ISDC_NODES_LOBATTO = 0, ISDC_NODES_RADAU_RIGHT = 1, ISDC_NODES_LEGENDRE = 2 };
/* Explicit part f^E of eq. (4): zero, u - u^3, or the viscous Burgers
 * advection -(d/dx + d/dy)(u^2/2) by a fifth-order WENO scheme (Jiang-Shu
 * weights, epsilon = 1e-6, local Lax-Friedrichs flux splitting with
 * alpha = max(|u_i|, |u_{i+1}|) per interface), conservative flux differences
 * (Sec. 4.1; periodic boundaries only). */
enum { ISDC_FE_ZERO = 0, ISDC_FE_CUBIC = 1, ISDC_FE_BURGERS = 2 };
/* Boundary conditions: homogeneous Dirichlet on (0, 1)^d with n = 2^k - 1
 * interior points per axis (h = 1/(n+1)), or periodic on [-1, 1)^d with
 * n = 2^k points per axis (h = 2/n; the Burgers setup of Sec. 4.1; compact
 * stencil, 2D, 2 <= k <= 13). */
enum { ISDC_BC_DIRICHLET = 0, ISDC_BC_PERIODIC = 1 };
/* Spatial discretisation of the Laplacian: the second-order (2d+1)-point
 * stencil (W = I, eq. (4)) or the fourth-order compact stencil with its
 * weighting matrix W (Sec. 3, eq. (5); 2D, weighted Jacobi with omega = 1,
 * warm-started V-cycles only). */
enum { ISDC_STENCIL_2ND = 0, ISDC_STENCIL_COMPACT4 = 1 };
/* Multigrid smoother: red-black Gauss-Seidel (red = even index sum, first) or
 * weighted Jacobi with omega = 2d/(2d+1) (omega = 1 with the compact stencil). */
enum { ISDC_SMOOTH_RBGS = 0, ISDC_SMOOTH_JACOBI = 1 };
/* Arithmetic of the V-cycles.  The SDC residual, the S*F quadrature, the
 * right-hand side and the node update are always float64. */
enum { ISDC_PREC_FP64 = 0, ISDC_PREC_MIXED = 1 /* float32 V-cycles */ };
/* Initial guess of each implicit solve (Sec. 4.3): u_{m+1}^k (the method),
 * or the two ablations the paper reports as failing: zero, or u_m^{k+1}. */
enum { ISDC_GUESS_PREV_SWEEP = 0, ISDC_GUESS_ZERO = 1, ISDC_GUESS_PREV_NODE = 2 };
/* Component operators for isdc_mg_op (parity and roofline probes). */
enum { ISDC_OP_SMOOTH = 0, ISDC_OP_RESTRICT = 1, ISDC_OP_PROLONG = 2, ISDC_OP_COARSE = 3,
       ISDC_OP_RESIDUAL_NORM = 4, ISDC_OP_EXPLICIT = 5 };

/* Kernels that isdc_time_kernel can time and isdc_probe_arm can follow
 * inside steps (see there). */
enum { ISDC_KERNEL_SMOOTH_RESTRICT = 0, ISDC_KERNEL_PROLONG_SMOOTH = 1, ISDC_KERNEL_SMOOTH = 2,
       ISDC_KERNEL_TAIL = 3, ISDC_KERNEL_QUAD = 4, ISDC_KERNEL_EXPLICIT = 5, ISDC_KERNEL_PROLONG_UPDATE = 6,
       ISDC_KERNEL_RESTRICT = 7, ISDC_KERNEL_RHS = 8, ISDC_KERNEL_ZSMOOTH_RESTRICT = 9 };

#define ISDC_MAX_M 9
#define ISDC_HIST 128

typedef struct {
    int32_t dim;      /* d = 1, 2 or 3                                                */
    int32_t n[3];     /* points per axis: Dirichlet 2^k - 1 interior points with      */
                      /* 1 <= k <= 15 (d = 1), k <= 13 (d = 2), k <= 10 (d = 3);      */
                      /* periodic 2^k with 2 <= k <= 13.  n[a] = 1 on the axes        */
                      /* a >= dim (else ISDC_E_INVAL); the used axes must have the    */
                      /* same count (else ISDC_E_UNSUPPORTED: the multigrid hierarchy */
                      /* coarsens every axis together)                                */
    double nu;        /* diffusion coefficient, finite and >= 0                       */
    int32_t fe_kind;  /* ISDC_FE_*                                                    */
    int32_t stencil;  /* ISDC_STENCIL_* (COMPACT4: dim = 2, smoother JACOBI, guess     */
                      /* PREV_SWEEP, not in batches; else ISDC_E_UNSUPPORTED)          */
    int32_t bc;       /* ISDC_BC_* (PERIODIC: stencil COMPACT4, n = 2^k, 2 <= k <= 13, */
                      /* not in batches; FE_BURGERS needs PERIODIC)                    */
} isdc_problem;

typedef struct {
    int32_t node_kind;   /* ISDC_NODES_*                                                   */
    int32_t M;           /* collocation nodes: 2..9 (Lobatto), 1..9 (right Radau, Legendre) */
    int32_t vcycles;     /* L V-cycles per implicit solve (Sec. 3); 0 = classical SDC:     */
                         /* cycle until the inner residual <= inner_tol (at most 100)      */
    double inner_tol;    /* max-norm inner residual tolerance (classical / early exit)     */
    int32_t early_exit;  /* 1: stop a solve before L cycles once inner_tol is met          */
    double sdc_tol;      /* > 0: stop once the max-norm SDC residual < sdc_tol (Sec. 3)    */
    int32_t max_sweeps;  /* 1..100000                                                      */
    int32_t smoother;    /* ISDC_SMOOTH_*                                                  */
    int32_t nu_pre;      /* pre-smoothing steps  (0..8)                                    */
    int32_t nu_post;     /* post-smoothing steps (0..8), nu_pre + nu_post >= 1             */
    int32_t precision;   /* ISDC_PREC_*                                                    */
    int32_t guess;       /* ISDC_GUESS_*                                                   */
    int32_t levels;      /* 1: ISDC (default); 2: two-level MLSDC with ISDC sweeps (Sec. 5):  */
                         /* each iteration is a fine sweep, one sweep on the (n-1)/2 grid   */
                         /* with the FAS term, and the coarse correction interpolated back  */
                         /* (second-order stencil, Dirichlet, n >= 3, not in batches)       */
} isdc_params;

typedef struct {
    int32_t sweeps;                    /* sweeps made in the last step (K~ of Sec. 3)     */
    int32_t hist_len;                  /* entries of residual_hist in use                 */
    int64_t vcycles;                   /* V-cycles over all implicit solves of the step   */
    double residual;                   /* last SDC residual                               */
    double residual_hist[ISDC_HIST];   /* residual after sweep 1, 2, ... (first 128)      */
    int64_t coarse_vcycles;            /* V-cycles of the coarse MLSDC level (levels = 2) */
} isdc_stats;

typedef struct isdc_plan isdc_plan;

/* Library version, major * 10000 + minor * 100 + patch. */
int isdc_version(void);

/* sizeof(isdc_problem), sizeof(isdc_params), sizeof(isdc_stats) as compiled
 * into the library, so that bindings can check their mirrors of the structs.
 * Host only; any pointer may be NULL. */
int isdc_abi_sizes(size_t* problem, size_t* params, size_t* stats);

/* Message of the last non-OK return on the calling thread ("" if none). */
const char* isdc_last_error(void);

/* Fill *p with the defaults: Lobatto, M = 3, L = 2, inner_tol = 1e-10,
 * early_exit = 0, sdc_tol = 1e-10, max_sweeps = 100, RB-GS V(1,1), FP64,
 * warm start from the previous sweep, one level.  Host only. */
int isdc_default_params(isdc_params* p);

/* Collocation tables (Sec. 2, eq. (1)-(2)), host only, float64:
 *   h_tau[j]      = tau_{j+1}, j = 0..M-1, nodes on [0, 1];
 *   h_Q[m*M + j]  = q_{m+1,j+1} = integral over [0, tau_{m+1}] of the Lagrange
 *                   polynomial l_{j+1} on tau_1..tau_M (may be NULL);
 *   h_S[m*M + j]  = s_{m,j+1} = q_{m+1,j+1} - q_{m,j+1} with q_0 = 0: the
 *                   node-to-node weights of eq. (2), m = 0..M-1 (may be NULL).
 * Arrays are owned by the caller (M, M*M, M*M doubles). */
int isdc_tables(int32_t node_kind, int32_t M, double* h_tau, double* h_Q, double* h_S);

/* Whole-step weights of the collocation rule (Sec. 1), host only, float64:
 * h_b[j] = integral over [0, 1] of l_{j+1} (M doubles, caller-owned).  They
 * give u(T_{n+1}) for Gauss-Legendre nodes; for the node families that end on
 * tau_M = 1 they equal the last row of Q. */
int isdc_end_weights(int32_t node_kind, int32_t M, double* h_b);

/* Bytes of device workspace a plan for (prob, par) needs (256-byte aligned
 * start required).  Host only. */
int isdc_workspace_bytes(const isdc_problem* prob, const isdc_params* par, size_t* out_bytes);

/* Create a plan over caller-owned device workspace d_workspace of `bytes`
 * bytes (at least isdc_workspace_bytes; 256-byte aligned).  The plan keeps
 * pointers into the workspace, which must outlive it.  Host only: no device
 * work is enqueued.  The plan binds to the HIP device current at its first
 * device call. */
int isdc_create(const isdc_problem* prob, const isdc_params* par, void* d_workspace,
                size_t bytes, isdc_plan** out_plan);

/* Destroy a plan (NULL is ignored).  Does not free the workspace. */
void isdc_destroy(isdc_plan* plan);

/* One ISDC time step (Sec. 2-3): d_u holds u_n (n^d float64) on entry and
 * u_{n+1} = u_M on return.  Sweeps run until the SDC residual < sdc_tol or
 * max_sweeps is reached.  Synchronises `stream` once per sweep to read the
 * 8-byte residual.  Returns ISDC_E_NOT_CONVERGED or ISDC_E_DIVERGED with the
 * last iterate in d_u and *out (may be NULL) filled. */
int isdc_step(isdc_plan* plan, double* d_u, double dt, void* stream, isdc_stats* out);

/* isdc_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same time step of (prob, par) on d_u, with the plan's workspace in a static
 * device array of the library (64 MiB, ISDC_STATIC_SCRATCH_BYTES; one copy per
 * device, held until the process ends) instead of a caller workspace.
 * Problems whose isdc_workspace_bytes exceed it return ISDC_E_WORKSPACE
 * before any device work.  The first call on a device looks up the array's
 * address and makes a host plan for that device; later calls allocate
 * nothing.  Results equal isdc_step's on a plan of the same (prob, par).
 * Every call on one device shares the array and that host plan, which keep
 * the last call's contents (nothing in them needs to start at zero): calls
 * that overlap on one device, from any thread or stream, race. */
#define ISDC_STATIC_SCRATCH_BYTES (64u << 20)
int isdc_step_noalloc(const isdc_problem* prob, const isdc_params* par, double* d_u, double dt, void* stream,
                      isdc_stats* out);

/* The pieces of isdc_step, for callers that drive sweeps themselves:
 * isdc_begin sets the initial iterate u_j^0 = u_0 at every node and computes
 * S*F(u^0).  d_u0 must stay valid and unchanged until isdc_end.
 * isdc_sweep makes one sweep of eq. (4) (with levels = 2: one MLSDC
 * iteration) and writes the new SDC residual to *h_residual (synchronises
 * `stream`).  isdc_end copies u_M to d_u_out (which may be d_u0). */
int isdc_begin(isdc_plan* plan, const double* d_u0, double dt, void* stream);
int isdc_sweep(isdc_plan* plan, void* stream, double* h_residual);
int isdc_end(isdc_plan* plan, double* d_u_out, void* stream);

/* Copy the current iterate at node j (1..M; 0 = u_0) to d_out (n^d float64). */
int isdc_node_values(isdc_plan* plan, int32_t j, double* d_out, void* stream);

/* Counters of the current / last step (sweeps, V-cycles, residual history). */
int isdc_get_stats(const isdc_plan* plan, isdc_stats* out);

/* `ncycles` V(nu_pre, nu_post)-cycles (the inner solver of Sec. 3) on
 * (I - c L_h) u = rhs, starting from the iterate in d_u and overwriting it.
 * precision selects float64 (ISDC_PREC_FP64: d_rhs, d_u are double*) or
 * float32 (ISDC_PREC_MIXED: float*).  c >= 0 is dt_m * nu.  If h_res_inf is
 * not NULL, max|rhs - (I - c L_h) u| after the cycles is written there and
 * `stream` is synchronised.  For a compact-stencil plan the operator here and
 * in isdc_mg_op is B_H = I + (h^2/12) L_H - c A_H on the level of spacing H
 * (h the finest spacing, so B_h = W - c A_h) and the smoother is weighted
 * Jacobi with omega = 1; on periodic grids coarse point I sits on fine point
 * 2I (n_l = n / 2^l) and indices wrap. */
int isdc_vcycle(isdc_plan* plan, double c, int32_t precision, const void* d_rhs, void* d_u,
                int32_t ncycles, void* stream, double* h_res_inf);

/* One multigrid component on level `level` (0 = finest, n_l = 2^(k-l) - 1),
 * for parity tests and kernel probes; precision as in isdc_vcycle.
 *   ISDC_OP_SMOOTH:        d_out <- one smoothing step of d_b on (I - c L) x = d_a
 *                          (d_out may equal d_b; d_a = rhs, d_b = iterate)
 *   ISDC_OP_RESTRICT:      d_out (level+1) <- full weighting of d_a - (I - c L) d_b
 *   ISDC_OP_PROLONG:       d_out (level)  += linear interpolation of d_a (level+1)
 *   ISDC_OP_COARSE:        d_out <- one V-cycle from zero for rhs d_a on this level
 *   ISDC_OP_RESIDUAL_NORM: *h_scalar <- max|d_a - (I - c L) d_b| (synchronises)
 *   ISDC_OP_EXPLICIT:      d_out <- f^E(d_a) on the finest grid, float64 (level 0,
 *                          c and precision ignored; plans with fe_kind
 *                          ISDC_FE_BURGERS, else ISDC_E_UNSUPPORTED)
 * Unused pointers may be NULL. */
int isdc_mg_op(isdc_plan* plan, int32_t op, int32_t level, double c, int32_t precision,
               const void* d_a, const void* d_b, void* d_out, void* stream, double* h_scalar);

/* Tile shapes of the multigrid kernels, one per level above the coarse tail
 * (level 0 = finest).  Shape 0 is the default tile (1D 1024, 2D 56x16, 3D
 * 32x8x4 points per workgroup), shapes 1 and 2 are smaller (1D 512 / 256,
 * 2D 56x8 / 24x8, 3D 16x8x4 / 16x4x4).  Every shape computes the same values
 * (the V-cycle of Sec. 3 is unchanged); only the launch shape differs.
 * On 3D levels of 127^3 and up, which run z-marching kernels (xy tiles of
 * 60x16 points in float32, 60x8 in float64), the shape picks the depth of a
 * workgroup's column of planes instead: shape 0 16 planes (4 on 127^3),
 * shape 2 8 (2), shape 1 the even depth at which every column of the level
 * fits in one round of resident workgroups of the kernel (its occupancy per
 * CU times the device's CUs).
 * isdc_autotune times the red-black kernels of every level with each shape
 * (three rounds of `reps` launches on `stream`, the fastest round of each
 * shape compared) and keeps the fastest; levels where the shape changes
 * nothing (Jacobi smoothing, compact stencil) keep shape 0.  It synchronises `stream`,
 * overwrites the plan's multigrid buffers, and is refused during a step.
 * The shapes, or a saved list, are read and written with the two calls
 * below; nlevels is the number of levels above the tail (*h_nlevels), and
 * h_shapes holds up to max_levels entries (caller-owned, may be NULL). */
int isdc_autotune(isdc_plan* plan, int32_t reps, void* stream, int32_t* h_shapes, int32_t max_levels,
                  int32_t* h_nlevels);
int isdc_set_tile_shapes(isdc_plan* plan, const int32_t* h_shapes, int32_t nlevels);
int isdc_get_tile_shapes(const isdc_plan* plan, int32_t* h_shapes, int32_t max_levels, int32_t* h_nlevels);

/* Time one of the plan's kernels as the step launches it: `reps` launches on
 * `stream`, back to back between one pair of HIP events (so the average
 * includes the short gap between consecutive launches but no per-launch
 * event cost), on the plan's own buffers at `level` (their contents are
 * whatever the last solve left; the timing does not depend on the values).
 * Writes the average duration per launch in microseconds to *h_avg_us and
 * the kernel's algorithmic bytes per launch (every array element read or
 * written once) to *h_bytes, and synchronises `stream`.  For measurement;
 * leaves the plan's workspace arrays with unspecified contents, so call it
 * only between steps.  Compact-stencil plans time ISDC_KERNEL_SMOOTH (the
 * V-cycle's launch of min(3, nu_pre) weighted-Jacobi steps of B fused with
 * the residual's full-weighting restriction; algorithmic bytes: the rhs and
 * the iterate read once, the iterate and the coarse rhs written once),
 * ISDC_KERNEL_TAIL (the compact tail) and ISDC_KERNEL_EXPLICIT only.
 *   ISDC_KERNEL_SMOOTH_RESTRICT  one red-black step fused with the residual's
 *                                full-weighting restriction (levels above the
 *                                coarse tail, d = 1 or 2; 3D levels of 127^3
 *                                and up)
 *   ISDC_KERNEL_PROLONG_SMOOTH   prolongation + correction + one red-black step
 *   ISDC_KERNEL_SMOOTH           one red-black step
 *   ISDC_KERNEL_TAIL             the single-workgroup coarse tail (level ignored)
 *   ISDC_KERNEL_QUAD             S*F quadrature + SDC residual of the current
 *                                iterate (a step must be in progress; level ignored)
 *   ISDC_KERNEL_EXPLICIT         the WENO5 Burgers advection of the finest grid
 *                                (ISDC_FE_BURGERS plans; level ignored)
 * precision selects the V-cycle arithmetic as in isdc_vcycle. */
int isdc_time_kernel(isdc_plan* plan, int32_t kernel, int32_t level, double c, int32_t precision, int32_t reps,
                     void* stream, double* h_avg_us, double* h_bytes);

/* In-step timing of one kernel, for measurement: after isdc_probe_arm, every
 * `every`-th launch (1..1000000) of `kernel` on multigrid level `level` that
 * the plan's steps make (isdc_step, isdc_sweep; level ignored for the
 * single-level kernels) records its own dispatch start and end into a HIP
 * event pair (hipExtLaunchKernelGGL, so no extra packet is placed between
 * launches), up to max_samples (1..1000000) launches.  The launches that are
 * followed (second-order stencil plans; other launches are not followed):
 *   ISDC_KERNEL_SMOOTH_RESTRICT  red-black step + residual + restriction
 *                                from a nonzero iterate (2D; 3D levels of
 *                                127^3 and up);
 *   ISDC_KERNEL_SMOOTH           a red-black step from a nonzero iterate;
 *   ISDC_KERNEL_ZSMOOTH_RESTRICT a red-black step from a zero iterate fused
 *                                with the residual's restriction (the first
 *                                launch of a V(1,1) cycle on a level that
 *                                starts from zero; 2D, and 3D levels of
 *                                127^3 and up);
 *   ISDC_KERNEL_RESTRICT         residual + full weighting (3D, Jacobi);
 *   ISDC_KERNEL_PROLONG_SMOOTH   prolongation + correction + red-black step;
 *   ISDC_KERNEL_PROLONG_UPDATE   the same fused with the node update
 *                                u = g + e (the last launch of a solve, level 0);
 *   ISDC_KERNEL_TAIL             the coarse tail;
 *   ISDC_KERNEL_QUAD             S*F quadrature + SDC residual (level 0);
 *   ISDC_KERNEL_RHS              the separate right-hand-side pass (level 0).
 * isdc_probe_read waits for the sampled launches' events, writes the number
 * of samples, their average duration in microseconds and their average
 * algorithmic bytes (every array element read or written once; the QUAD
 * figure depends on how many node arrays the sampled launches read), and
 * disarms the probe.  Host only, apart from that wait; arming again restarts
 * the sample.  Event pairs are created by the arming call and kept by the
 * plan. */
int isdc_probe_arm(isdc_plan* plan, int32_t kernel, int32_t level, int32_t every, int32_t max_samples);
int isdc_probe_read(isdc_plan* plan, int64_t* h_samples, double* h_avg_us, double* h_bytes);

/* ---------------------------------------------------------------- batches
 * A batch advances many independent ISDC instances ("slots") together: every
 * phase of a sweep is one kernel launch covering all running slots, so small
 * and uneven instances fill the GPU together.  Slots may differ in grid size,
 * nu, f^E, dt, node family, M, tolerance, max_sweeps, number of steps and
 * (2D) cycles; all slots of a batch share the dimension, the V-cycle
 * precision and L, and run red-black Gauss-Seidel V(1,1) cycles or, in 2D,
 * weighted-Jacobi V(nu1, nu2) cycles with 1 <= nu1, nu2 <= 3, warm-started
 * from the previous sweep (Sec. 3, Sec. 4.3) -- other parameters return
 * ISDC_E_UNSUPPORTED.  A slot's results are bitwise those of isdc_step on the
 * same instance. */
typedef struct isdc_batch isdc_batch;

/* Slot states reported by isdc_batch_slot_info. */
enum { ISDC_SLOT_FREE = 0, ISDC_SLOT_RUNNING = 1, ISDC_SLOT_FINISHED = 2 };

/* ---- Fixed instances, one full time step per call.
 * `count` (1..4096) independent instances (Sec. 2, eq. (1)-(4): each its own
 * u_0, f^I/f^E split, nodes and M, and L V-cycles per solve), probs[i] and
 * pars[i] for instance i; all must share dim, precision and L >= 1, and run
 * the batch's solver (above).  isdc_batch_bytes gives the device workspace
 * of such a batch: the batch's own arrays followed by every instance's plan
 * workspace.  Host only; probs and pars are copied. */
int isdc_batch_bytes(int32_t count, const isdc_problem* probs, const isdc_params* pars, size_t* out_bytes);
int isdc_batch_create(int32_t count, const isdc_problem* probs, const isdc_params* pars, void* d_workspace,
                      size_t bytes, isdc_batch** out);

/* One ISDC time step of every active instance (active[i] != 0; active NULL =
 * all): d_u[i] (instance i's n^d float64 state) holds u_n on entry and
 * u_{n+1} on return, dt[i] > 0 is its step.  All active instances sweep
 * together (one launch per sweep phase, one 8-byte-per-instance residual
 * read-back per sweep) until each has converged or stopped; stats[i] (stats
 * may be NULL; entries of inactive instances are untouched) receives its
 * counters.  Instance i's result is bitwise that of isdc_step on its own plan.
 * Returns ISDC_OK if every active instance converged, else the status of the
 * first one (by index) that did not (ISDC_E_NOT_CONVERGED / ISDC_E_DIVERGED),
 * with every active d_u[i] holding that instance's last iterate.  Invalid
 * pointers or dt are rejected before any device work.  Synchronises `stream`.
 * Only for batches made by isdc_batch_create. */
int isdc_batch_step(isdc_batch* batch, double* const* d_u, const double* dt, const int32_t* active, void* stream,
                    isdc_stats* stats);

/* ---- Open slots, for continuous batching (a serving loop).
 * isdc_batch_workspace_bytes: device workspace of a slot batch with
 * `capacity` slots (1..4096): slot descriptors, states, residuals and launch
 * maps.  Host only. */
int isdc_batch_workspace_bytes(int32_t capacity, size_t* out_bytes);

/* Open a slot batch over caller-owned device workspace (256-byte aligned, at
 * least isdc_batch_workspace_bytes).  dim, precision (ISDC_PREC_*) and
 * vcycles (L >= 1) are common to all slots.  Host only. */
int isdc_batch_open(int32_t capacity, int32_t dim, int32_t precision, int32_t vcycles, void* d_workspace,
                    size_t bytes, isdc_batch** out);

/* Destroy a batch (NULL is ignored); frees its slot plans and pinned host
 * staging, not the caller's workspaces. */
void isdc_batch_destroy(isdc_batch* batch);

/* Occupy a slot that is not running: the instance (prob, par) over its own
 * plan workspace d_plan_workspace (>= isdc_workspace_bytes(prob, par) bytes,
 * 256-byte aligned), state d_u (n^d float64: u_0 on entry, u after the last
 * step when the slot finishes; it must stay valid until then), step size dt
 * and nsteps >= 1 steps.  The slot starts at the next isdc_batch_advance.
 * Host only. */
int isdc_batch_set(isdc_batch* batch, int32_t slot, const isdc_problem* prob, const isdc_params* par,
                   void* d_plan_workspace, size_t plan_bytes, double* d_u, double dt, int32_t nsteps);

/* One sweep of every running slot (slots that start a step are initialised
 * first).  Synchronises `stream` once to read one residual per slot; a slot
 * whose step converged (residual < sdc_tol) writes u_M to its state and
 * either starts its next step at the next call or finishes; a slot whose
 * residual is non-finite or that reaches max_sweeps finishes with
 * ISDC_E_DIVERGED / ISDC_E_NOT_CONVERGED and its last iterate written.  Other
 * slots are not affected.  *h_running (may be NULL) receives the number of
 * slots still running. */
int isdc_batch_advance(isdc_batch* batch, void* stream, int32_t* h_running);

/* Measurement of the batch sweep's launch schedule: `reps` more sweeps of
 * the running slots (every one of which must have started its step, i.e. the
 * batch was advanced once), either launched one kernel at a time as
 * isdc_batch_advance does (graph = 0) or captured once into a HIP graph and
 * replayed (graph = 1; `stream` must not be the null stream).  Writes the
 * average microseconds per sweep (HIP events on `stream`) and the kernel
 * launches per sweep; makes no decisions and leaves the running slots' states
 * unspecified, so re-set the slots afterwards.  Synchronises `stream`. */
int isdc_batch_time_sweeps(isdc_batch* batch, int32_t reps, int32_t graph, void* stream, double* h_us_per_sweep,
                           int32_t* h_launches);

/* State (ISDC_SLOT_*), status of a finished slot, steps completed and the
 * statistics of its last completed step.  Host only; outputs may be NULL. */
int isdc_batch_slot_info(const isdc_batch* batch, int32_t slot, int32_t* state, int32_t* status,
                         int32_t* steps_done, isdc_stats* last_step);

/* Free a slot (finished or not) for reuse.  Host only. */
int isdc_batch_release(isdc_batch* batch, int32_t slot);

#ifdef __cplusplus
}
#endif

#endif /* ISDC_H */
