// Host-side plan structure and error plumbing shared by the runtime and the
// batch engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

namespace isdc {

std::string& last_error();

#define HIPCHK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            throw ::isdc::Error{ISDC_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
    } while (0)

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
inline size_t pow_d(size_t n, int d) { return d == 1 ? n : (d == 2 ? n * n : n * n * n); }

// Run f, turning exceptions into a status code and the thread's last error.
template <typename F>
int guarded(F&& f) {
    try {
        f();
        last_error().clear();
        return ISDC_OK;
    } catch (const Error& e) {
        last_error() = e.msg;
        return e.code;
    } catch (const std::exception& e) {
        last_error() = e.what();
        return ISDC_E_HIP;
    } catch (...) {
        last_error() = "unknown error";
        return ISDC_E_HIP;
    }
}

struct Level {
    int n;
    double h;
    size_t N;
    void* r;
    void* e;
    void* e2;  // ping-pong partner of the out-of-place smoothers
    int shape = 0;  // tile shape of the tiled kernels on this level (isdc_autotune)
};

// In-step timing of one kernel kind on one level (isdc_probe_arm /
// isdc_probe_read): every `every`-th matching launch records its dispatch
// start and end into the next event pair of the pool.
struct ProbeState {
    int kind = -1;   // ISDC_KERNEL_* (-1: off)
    int level = 0;
    int every = 1;
    int64_t seen = 0;       // matching launches since arming
    size_t used = 0;        // event pairs handed out
    size_t limit = 0;       // at most this many samples
    double bytes = 0.0;     // algorithmic bytes of the sampled launches
    std::vector<LaunchProbe> pool;
};

// Per-sweep host trace (environment variable ISDC_TRACE, read once): unset,
// empty or "0" = off; "1" or "stderr" = standard error; otherwise a file path
// the lines are appended to.  nullptr when off.
FILE* trace_stream();

void validate(const isdc_problem* pb, const isdc_params* pr);
size_t layout(const isdc_problem& pb, const isdc_params& pr, char* base, isdc_plan* p);

}  // namespace isdc

struct isdc_plan {
    isdc_problem prob;
    isdc_params par;
    int d, n;
    size_t N;
    double h;
    int M;
    double tau[ISDC_MAX_M], Q[ISDC_MAX_M * ISDC_MAX_M], S[ISDC_MAX_M * ISDC_MAX_M];
    double dtau[ISDC_MAX_M];  // tau_{m+1} - tau_m, tau_0 = 0
    double b[ISDC_MAX_M];     // whole-step weights (end value of Gauss-Legendre steps)
    bool end_quad = false;    // Gauss-Legendre: u_{n+1} by the end-point quadrature
    double* END = nullptr;    // dt sum_j b_j f_j of the final iterate (end_quad only)
    isdc::MGConfig mg;
    std::vector<isdc::Level> lev;
    int tail;  // index of the level run by the single-workgroup tail kernel

    double* U[2][ISDC_MAX_M + 1];  // node arrays written by sweeps (index 0 unused)
    double* SF[ISDC_MAX_M];        // S_m^{m+1} F for substep m (NULL if dt_m = 0)
    double* partial;
    double* scalars;

    // compact stencil (eq. (5)): B = W - c A_h, weighted Jacobi; W inverted
    // for the residual by Chebyshev iteration
    bool compact = false;
    bool periodic = false;         // [-1, 1)^2 with n = 2^k points per axis, h = 2 / n
    double w = 0.0;                // h^2 / 12
    double* Yq[ISDC_MAX_M];        // dt Q_m F~ per node m+1 (NULL: node with Q row 0)
    double* X[ISDC_MAX_M];         // W^{-1} Yq[m], warm start of the next sweep's solve
    double* WX = nullptr;          // W solve: partner of the iterate's ping-pong
    double* WD[2] = {nullptr, nullptr};  // W solve: Chebyshev direction, double-buffered
    bool x_valid = false;
    // stencil f^E (WENO5 Burgers): f^E of u_0 and of every node array
    bool fe_arrays = false;
    double* FE0 = nullptr;
    double* FEU[2][ISDC_MAX_M + 1];  // f^E(U[w][j]) (NULL where U[w][j] is)

    // two-level MLSDC (levels = 2): coarse node values R U_j (index 0: R u_0),
    // the coarse sweep's new values, and the injected S F of the fine level
    int levels = 1;
    double* Rf[ISDC_MAX_M + 1];
    double* Uc[ISDC_MAX_M + 1];
    double* SFc[ISDC_MAX_M];

    // step state
    const double* u0 = nullptr;
    double dt = 0.0;
    const double* cur[ISDC_MAX_M + 1];  // current iterate per node (0 = u_0)
    const double* curfe[ISDC_MAX_M + 1];  // f^E of cur[j] (fe_arrays only)
    int wbuf = 0;                       // which U table the next sweep writes
    bool begun = false;
    isdc_stats stats;
    double* h_pinned = nullptr;
    isdc::ProbeState probe;
    // device-side inner stopping test: cycles each substep needed in its last
    // solve and in the first sweep of the last step (0: none yet), and the
    // substep being solved
    int gate_hint[ISDC_MAX_M] = {0};
    int gate_hint_first[ISDC_MAX_M] = {0};
    int gate_substep = 0;
};

namespace isdc {
// Fill a freshly allocated plan from validated arguments (host only).
void init_plan(isdc_plan* p, const isdc_problem* prob, const isdc_params* par, void* d_workspace);
}  // namespace isdc
