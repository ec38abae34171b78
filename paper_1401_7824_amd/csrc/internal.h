// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "../../include/isdc.h"
#include "tables.h"

namespace isdc {

// ---------------------------------------------------------------- errors
struct Error {
    int code;
    std::string msg;
};

// ---------------------------------------------------------------- in-step launch timing
// An event pair that one launch records its own dispatch start and end into
// (hipExtLaunchKernelGGL).  The runtime arms one on the calling thread right
// before a launcher call it wants timed and disarms it after; the first
// ISDC_LAUNCH inside the launcher consumes it.
struct LaunchProbe {
    hipEvent_t start, stop;
};
LaunchProbe*& armed_probe();

#define ISDC_LAUNCH(kernel, grid, block, shmem, stream, ...)                                              \
    do {                                                                                                  \
        ::isdc::LaunchProbe* probe_ = ::isdc::armed_probe();                                              \
        if (probe_) {                                                                                     \
            ::isdc::armed_probe() = nullptr;                                                              \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, probe_->start, probe_->stop, 0,     \
                                  __VA_ARGS__);                                                           \
        } else {                                                                                          \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                          \
        }                                                                                                 \
    } while (0)

// Device-side gate of a solve's V-cycles (classical SDC / early exit): while
// the runtime has set a gate on the calling thread, the multigrid launchers
// pass it to their kernels as the last argument (ISDC_GLAUNCH), and each
// kernel returns at once when gate[0] != 0 -- set on the device by
// launch_reduce_gate once the inner residual meets its tolerance -- so a
// whole run of cycles can be enqueued before the host looks at the result.
const int*& current_gate();

#define ISDC_GLAUNCH(kernel, grid, block, shmem, stream, ...) \
    ISDC_LAUNCH(kernel, grid, block, shmem, stream, __VA_ARGS__, ::isdc::current_gate())

// ---------------------------------------------------------------- multigrid launchers
// Coefficients of A_l = I - c L_{h_l} on one level: a = c / h_l^2,
// diag = 1 + 2 d a, invdiag = 1 / diag, w = Jacobi weight.
template <typename T>
struct Coef {
    T a, diag, invdiag, w;
};

// Level coefficients of the coarse tail (level 0 = the tail's finest level),
// computed on the host exactly as make_coef does.
struct TailCoefs {
    double a[16], diag[16], invdiag[16];
};

struct MGConfig {
    int d;
    int smoother;  // ISDC_SMOOTH_*
    int nu_pre, nu_post;
    double omega;  // Jacobi weight
};

template <typename T>
Coef<T> make_coef(double c, double h, int d, double omega);

// One smoothing step.  RB-GS works in place on `u` (u_in is ignored unless
// zero_guess is false and u_in != u, in which case it is copied first by the
// caller); Jacobi writes u_out from u_in.  zero_guess: the current iterate is
// identically zero and is not read.
template <typename T>
hipError_t launch_smooth(const MGConfig& cfg, int n, const Coef<T>& co, bool zero_guess,
                         const T* rhs, const T* u_in, T* u_out, hipStream_t s);

// rc = full weighting of (rhs - A u) on the fine level with n points per axis.
template <typename T>
hipError_t launch_restrict(int d, int n, const Coef<T>& co, const T* rhs, const T* u, T* rc,
                           hipStream_t s);

// u += linear interpolation of ec (fine level n points per axis).
template <typename T>
hipError_t launch_prolong(int d, int n, const T* ec, T* u, hipStream_t s);

// One complete V-cycle on a small level (n <= tail_max_n(d)) and every level
// below it, in a single workgroup.  zero_guess: start from e = 0, otherwise
// from the iterate in e.
template <typename T>
hipError_t launch_tail(const MGConfig& cfg, int n, double c, double h, bool zero_guess, const T* rhs, T* e,
                       hipStream_t s);
int tail_max_n(int d);

// Tiled kernels (mg_tiles.hip).  One complete red-black Gauss-Seidel step
// from e_in to e_out (e_out != e_in; zero: e_in is identically zero and is
// not read).
// `shape` selects the tile shape of the tiled kernels, or the column depth of
// the z-marching kernels on 3D levels of 127^3 and up (0 .. kTileShapes - 1;
// 0 = the default); every shape computes the same values.
constexpr int kTileShapes = 3;
template <typename T>
hipError_t launch_rbgs_tile(int d, int n, const Coef<T>& co, bool zero, const T* r, const T* e_in, T* e_out,
                            hipStream_t s, int shape = 0);
// rc = full weighting of (r - A e); rc has (n-1)/2 points per axis.
template <typename T>
hipError_t launch_restrict_tile(int d, int n, const Coef<T>& co, const T* r, const T* e, T* rc, hipStream_t s);
// One red-black step from e_in to e_out fused with rc = full weighting of
// (r - A e_out).  d = 1, 2, and 3D z-marched levels (rbgs_restrict_fused
// says which).
bool rbgs_restrict_fused(int d, int n);
template <typename T>
hipError_t launch_rbgs_restrict_tile(int d, int n, const Coef<T>& co, bool zero, const T* r, const T* e_in, T* e_out,
                                     T* rc, hipStream_t s, int shape = 0);
// e_in + P ec followed by one red-black step.  mode 0: result to e_out;
// mode 1: u_out = g + result (float64); mode 2: u_out = result.
template <typename T>
hipError_t launch_prolong_rbgs_tile(int d, int n, const Coef<T>& co, const T* r, const T* e_in, const T* ec,
                                    T* e_out, const double* g, double* u_out, int mode, hipStream_t s,
                                    int shape = 0);

// partial[b] = max |rhs - A u| over the points of block b; returns the block
// count in *nblocks (<= kReduceBlocks).
constexpr int kReduceBlocks = 1024;
template <typename T>
hipError_t launch_resnorm(int d, int n, const Coef<T>& co, const T* rhs, const T* u,
                          double* partial, int* nblocks, hipStream_t s);

// out[0] = NaN-propagating max of partial[0..nblocks).
hipError_t launch_reduce_max(const double* partial, int nblocks, double* out, hipStream_t s);

// gate[0] = gate[1] = 0 (a kernel, not a memset).
hipError_t launch_gate_reset(int* gate, hipStream_t s);
// The inner stopping test on the device: unless gate[0] is set, res = max of
// partial[0..nblocks) goes to *res_out, and gate[0] = 1 if res <= tol (Sec. 3:
// the classical solve stops once its residual meets the inner tolerance) or
// gate[1] >= limit; otherwise, if count_cycle, gate[1] += 1 (the cycle that
// follows this test runs).
hipError_t launch_reduce_gate(const double* partial, int nblocks, double tol, int limit, int count_cycle, int* gate,
                              double* res_out, hipStream_t s);

template <typename T>
hipError_t launch_fill(T* p, size_t count, T value, hipStream_t s);

template <typename T>
hipError_t launch_copy(const T* src, T* dst, size_t count, hipStream_t s);

// ---------------------------------------------------------------- SDC launchers
struct QuadArgs {
    const double* u[ISDC_MAX_M + 1];    // u[0] = u_0, u[j] = node j (j = 1..M)
    double* sf[ISDC_MAX_M];             // S*F for substep m (NULL: not written)
    double dtS[ISDC_MAX_M * ISDC_MAX_M];  // dt * s_{m,j}
    double dtQ[ISDC_MAX_M * ISDC_MAX_M];  // dt * q_{m,j}
    double nu_h2;                       // nu / h^2
    int M;
    int n;
    int fe;
};

// For every point: f_j = nu L_h u_j + f^E(u_j); sf[m] = sum_j dt s_{m,j} f_j;
// partial[b] = max over the block of |u_0 + sum_j dt q_{m,j} f_j - u_m|.
// partial must hold quad_partials(d, n) entries.
int quad_partials(int d, int n);
hipError_t launch_quad_residual(int d, const QuadArgs& qa, double* partial, int* nblocks,
                                hipStream_t s);

struct RhsArgs {
    const double* um_new;  // u_m^{k+1}
    const double* um_old;  // u_m^k
    const double* up_old;  // u_{m+1}^k
    const double* sf;      // S_m^{m+1} F(u^k)
    double dtm;            // dt_m
    double c;              // dt_m nu
    double nu_h2;          // nu / h^2
    int n;
    int fe;
    int guess;             // ISDC_GUESS_*
};

// r = rhs - (I - c L_h) g for the right-hand side of eq. (4) and the guess g.
template <typename T>
hipError_t launch_euler_rhs(int d, const RhsArgs& ra, T* r, hipStream_t s);
// launch_euler_rhs (guess ISDC_GUESS_PREV_SWEEP) followed by the zero-start
// launch_rbgs_restrict_tile on a 2D level, in one launch: r, e_out and rc
// receive the same values.
template <typename T>
hipError_t launch_rhs_rbgs_restrict_tile(int d, int n, const RhsArgs& ra, const Coef<T>& co, T* r, T* e_out, T* rc,
                                         hipStream_t s, int shape = 0);

// u_out = g + e with g = u_{m+1}^k (PREV_SWEEP), 0 (ZERO) or u_m^{k+1} (PREV_NODE).
template <typename T>
hipError_t launch_node_update(size_t N, int guess, const double* up_old, const double* um_new,
                              const T* e, double* u_out, hipStream_t s);

// ---------------------------------------------------------------- two-level MLSDC (mlsdc.hip)
// coarse[I] = fine[2I+1] per axis (fine n = 2^k - 1 points, coarse (n-1)/2).
hipError_t launch_inject(int d, int n, const double* fine, double* coarse, hipStream_t s);
// u += cubic interpolation of (coarse_new - coarse_old) onto the fine grid of n points.
hipError_t launch_cubic_correct(int d, int n, const double* coarse_new, const double* coarse_old, double* u,
                                hipStream_t s);

// ---------------------------------------------------------------- compact stencil (2D, compact.hip)
// B_H = I + w L_H - c A_H on a level of spacing H: centre b0, the 4 edge
// neighbours bf, the 4 corners bc; omega of the weighted-Jacobi smoother.
template <typename T>
struct CCoef {
    T b0, bf, bc, inv_b0, omega;
};
template <typename T>
CCoef<T> make_ccoef(double c, double w, double H, double omega);

struct CTailCoefs {
    double b0[16], bf[16], bc[16];
};

struct CRhsArgs {
    const double* um_new;  // u_m^{k+1}
    const double* um_old;  // u_m^k
    const double* up_old;  // u_{m+1}^k (the guess)
    const double* sf;      // S_m^{m+1} F~(u^k)
    double dtm;
    int n;
    int fe;
    const double* fe_new;  // f^E(u_m^{k+1}) and f^E(u_m^k) as arrays (stencil f^E), or NULL:
    const double* fe_old;  // then f^E is evaluated pointwise from fe
};

struct CQuadArgs {
    const double* u[ISDC_MAX_M + 1];  // u_0 .. u_M
    const double* feu[ISDC_MAX_M + 1];  // f^E(u_j) as arrays (stencil f^E), or NULL: pointwise
    double* sf[ISDC_MAX_M];           // S_m^{m+1} F~ (NULL: not needed)
    double* y[ISDC_MAX_M];            // dt Q_m F~    (NULL: not needed)
    double dtS[ISDC_MAX_M * ISDC_MAX_M];
    double dtQ[ISDC_MAX_M * ISDC_MAX_M];
    double nu_6h2;                    // nu / (6 h^2)
    int n, fe, M;
};

constexpr int kCResBlocks = 256;
constexpr int kCTailMaxPeriodic = 32;  // largest periodic level of the compact tail
struct CResArgs {
    const double* u0;
    const double* um[ISDC_MAX_M];  // u_m of the nodes taking part
    const double* xm[ISDC_MAX_M];  // W^{-1} Y_m of the same nodes
    size_t N;
    int count;
};

// Compact-stencil launchers; per selects periodic wrap-around (n = 2^k,
// coarse n/2) instead of zero Dirichlet ghosts (n = 2^k - 1, coarse (n-1)/2).
// One weighted-Jacobi step e_out = e + omega (r - B e) / b0 (zero: e = 0).
template <typename T>
hipError_t launch_cjacobi(int n, const CCoef<T>& k, bool zero, const T* r, const T* e_in, T* e_out, bool per,
                          hipStream_t s);
// nsteps (1..3) weighted-Jacobi steps from e_in to e_out in one launch (the
// result of nsteps single steps); zero: e_in is zero and not read.
template <typename T>
hipError_t launch_cjacobi_steps(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out,
                                bool per, hipStream_t s);
// nsteps (1..3) Jacobi steps from e_in to e_out fused with rc = full
// weighting of r - B e_out on the next coarser level (zero: e_in is zero).
template <typename T>
hipError_t launch_cjres(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out, T* rc,
                        bool per, hipStream_t s);
// e_in + P ec (linear interpolation of the coarse correction) followed by
// nsteps (1..3) Jacobi steps, into e_out.
// The fused row-tile Jacobi kernels above for the second-order five-point
// operator I - c L_h on a 2D Dirichlet level (k from make_coef5): nsteps
// (1..3) weighted-Jacobi steps; the same fused with the residual's full
// weighting into rc; the prolongation + correction fused with nsteps steps.
template <typename T>
CCoef<T> make_coef5(double c, double h, double omega);
template <typename T>
hipError_t launch_jacobi5_steps(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out,
                                hipStream_t s);
template <typename T>
hipError_t launch_jres5(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out, T* rc,
                        hipStream_t s);
// u_out != NULL: the result is not written to e_out; u_out = g + result (float64).
template <typename T>
hipError_t launch_pjac5(int n, const CCoef<T>& k, int nsteps, const T* r, const T* e_in, const T* ec, T* e_out,
                        const double* g, double* u_out, hipStream_t s);
template <typename T>
hipError_t launch_cpjac(int n, const CCoef<T>& k, int nsteps, const T* r, const T* e_in, const T* ec, T* e_out,
                        bool per, hipStream_t s);
// rc = full weighting of r - B e on the next coarser level.
template <typename T>
hipError_t launch_cresfw(int n, const CCoef<T>& k, const T* r, const T* e, T* rc, bool per, hipStream_t s);
// u += periodic linear interpolation of ec ((n/2)^2 -> n^2).
template <typename T>
hipError_t launch_cprolong_p(int n, const T* ec, T* u, hipStream_t s);
// Per-block maxima of |r - B e| in partial[0 .. *nblocks).
template <typename T>
hipError_t launch_cresnorm(int n, const CCoef<T>& k, const T* r, const T* e, double* partial, int* nblocks, bool per,
                           hipStream_t s);
// r = W [u_m^{k+1} - g + dt_m (f^E(u_m^{k+1}) - f^E(u_m^k))] + S_m F~.
template <typename T>
hipError_t launch_crhs(const CRhsArgs& a, T* out, bool per, hipStream_t s);
// S F~ and dt Q F~ of the current node values.
hipError_t launch_cquad(const CQuadArgs& a, int M, bool per, hipStream_t s);
// Per-node maxima of |u_0 + x_m - u_m|; kCResBlocks * count partials.
hipError_t launch_cres(const CResArgs& a, double* partial, int* nblocks, hipStream_t s);
// out = the periodic WENO5 Burgers advection -div(u^2/2) of u (n^2, spacing h).
hipError_t launch_weno_burgers(int n, double h, const double* u, double* out, hipStream_t s);
// One Chebyshev step for W x = y on the finest 2D grid (W = I + (h^2/12) L_h):
// kind 0 = first step from zero, 1 = first step from x_in, 2 = later step with
// coefficients cd, cr; x_out and x_in must differ, d is updated in place.
hipError_t launch_wcheb(int n, bool per, int kind, const double* y, const double* x_in, double* x_out, double* d,
                        double cd, double cr, hipStream_t s);
// kWChebSteps Chebyshev steps in one launch (the result of that many single
// steps): kind as above for the first step, cd[k], cr[k] the coefficients of
// step k (those of a first step are not used); d goes from d_in to d_out
// (d_in != d_out), x from x_in to x_out.
constexpr int kWChebSteps = 4;
hipError_t launch_wcheb_steps(int n, bool per, int kind, int nsteps, const double* y, const double* x_in,
                              double* x_out, const double* d_in, double* d_out, const double* cd, const double* cr,
                              hipStream_t s);
// One V-cycle of B (weighted Jacobi V(nu_pre, nu_post)) on a level of at
// most 63^2 (Dirichlet) or 32^2 (periodic) points in one workgroup.
template <typename T>
hipError_t launch_ctail(const MGConfig& mg, int n, double c, double w, double h, bool zero, const T* rhs, T* e,
                        bool per, hipStream_t s);

}  // namespace isdc
