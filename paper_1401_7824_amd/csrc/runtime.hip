// Host runtime and C ABI of libisdc: plan layout over the caller's device
// workspace, the V-cycle schedule, the SDC sweep of eq. (4) and the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"

using namespace isdc;

namespace isdc {
std::string& last_error() {
    thread_local std::string msg;
    return msg;
}
FILE* trace_stream() {
    static FILE* const stream = [] () -> FILE* {
        const char* v = std::getenv("ISDC_TRACE");
        if (!v || !*v || std::strcmp(v, "0") == 0) return nullptr;
        if (std::strcmp(v, "1") == 0 || std::strcmp(v, "stderr") == 0) return stderr;
        FILE* f = std::fopen(v, "a");
        return f ? f : stderr;
    }();
    return stream;
}
const int*& current_gate() {
    thread_local const int* gate = nullptr;
    return gate;
}
LaunchProbe*& armed_probe() {
    thread_local LaunchProbe* probe = nullptr;
    return probe;
}
}  // namespace isdc

namespace {

bool valid_n(int d, int n) {
    if (n < 1 || ((n + 1) & n) != 0) return false;
    int k = 0;
    while ((1 << k) - 1 < n) ++k;
    int kmax = d == 1 ? 15 : (d == 2 ? 13 : 10);
    return k <= kmax;
}

}  // namespace

void isdc::validate(const isdc_problem* pb, const isdc_params* pr) {
    if (!pb || !pr) fail(ISDC_E_INVAL, "NULL problem or params");
    if (pb->dim < 1 || pb->dim > 3) fail(ISDC_E_INVAL, "dim must be 1, 2 or 3");
    if (pb->bc != ISDC_BC_DIRICHLET && pb->bc != ISDC_BC_PERIODIC) fail(ISDC_E_INVAL, "unknown bc");
    for (int a = pb->dim; a < 3; ++a)
        if (pb->n[a] != 1) fail(ISDC_E_INVAL, "n[a] must be 1 on the axes a >= dim");
    for (int a = 1; a < pb->dim; ++a)
        if (pb->n[a] != pb->n[0]) fail(ISDC_E_UNSUPPORTED, "grids must have the same number of points on every axis");
    if (pb->bc == ISDC_BC_PERIODIC) {
        if (pb->n[0] < 4 || pb->n[0] > 8192 || (pb->n[0] & (pb->n[0] - 1)) != 0)
            fail(ISDC_E_INVAL, "periodic grids need n = 2^k points with 2 <= k <= 13");
    } else if (!valid_n(pb->dim, pb->n[0])) {
        fail(ISDC_E_INVAL, "n must be 2^k - 1 within the size limit for dim");
    }
    if (!std::isfinite(pb->nu) || pb->nu < 0) fail(ISDC_E_INVAL, "nu must be finite and >= 0");
    if (pb->fe_kind != ISDC_FE_ZERO && pb->fe_kind != ISDC_FE_CUBIC && pb->fe_kind != ISDC_FE_BURGERS)
        fail(ISDC_E_INVAL, "unknown fe_kind");
    if (pr->node_kind == ISDC_NODES_LOBATTO) {
        if (pr->M < 2 || pr->M > ISDC_MAX_M) fail(ISDC_E_INVAL, "Gauss-Lobatto needs 2 <= M <= 9");
    } else if (pr->node_kind == ISDC_NODES_RADAU_RIGHT) {
        if (pr->M < 1 || pr->M > ISDC_MAX_M) fail(ISDC_E_INVAL, "right Gauss-Radau needs 1 <= M <= 9");
    } else if (pr->node_kind == ISDC_NODES_LEGENDRE) {
        if (pr->M < 1 || pr->M > ISDC_MAX_M) fail(ISDC_E_INVAL, "Gauss-Legendre needs 1 <= M <= 9");
    } else {
        fail(ISDC_E_INVAL, "unknown node_kind");
    }
    if (pr->vcycles < 0 || pr->vcycles > 64) fail(ISDC_E_INVAL, "vcycles must be in 0..64");
    if (!std::isfinite(pr->inner_tol) || pr->inner_tol < 0) fail(ISDC_E_INVAL, "inner_tol must be finite, >= 0");
    if (pr->early_exit != 0 && pr->early_exit != 1) fail(ISDC_E_INVAL, "early_exit must be 0 or 1");
    // the sweeps stop once the residual is strictly below sdc_tol (Sec. 3), which a zero tolerance never allows
    if (!std::isfinite(pr->sdc_tol) || pr->sdc_tol <= 0) fail(ISDC_E_INVAL, "sdc_tol must be finite and > 0");
    if (pr->max_sweeps < 1 || pr->max_sweeps > 100000) fail(ISDC_E_INVAL, "max_sweeps must be in 1..100000");
    if (pr->smoother != ISDC_SMOOTH_RBGS && pr->smoother != ISDC_SMOOTH_JACOBI) fail(ISDC_E_INVAL, "unknown smoother");
    if (pr->nu_pre < 0 || pr->nu_pre > 8 || pr->nu_post < 0 || pr->nu_post > 8 || pr->nu_pre + pr->nu_post < 1)
        fail(ISDC_E_INVAL, "nu_pre, nu_post must be in 0..8 with nu_pre + nu_post >= 1");
    if (pr->precision != ISDC_PREC_FP64 && pr->precision != ISDC_PREC_MIXED) fail(ISDC_E_INVAL, "unknown precision");
    if (pr->guess < ISDC_GUESS_PREV_SWEEP || pr->guess > ISDC_GUESS_PREV_NODE) fail(ISDC_E_INVAL, "unknown guess");
    if (pb->stencil != ISDC_STENCIL_2ND && pb->stencil != ISDC_STENCIL_COMPACT4) fail(ISDC_E_INVAL, "unknown stencil");
    if (pb->stencil == ISDC_STENCIL_COMPACT4) {
        if (pb->dim != 2) fail(ISDC_E_UNSUPPORTED, "the compact stencil is implemented in 2D");
        if (pr->smoother != ISDC_SMOOTH_JACOBI)
            fail(ISDC_E_UNSUPPORTED, "the compact stencil needs the Jacobi smoother (red-black is not Gauss-Seidel for 9 points)");
        if (pr->guess != ISDC_GUESS_PREV_SWEEP)
            fail(ISDC_E_UNSUPPORTED, "the compact stencil warm-starts from the previous sweep only");
    }
    if (pr->levels != 1 && pr->levels != 2) fail(ISDC_E_INVAL, "levels must be 1 or 2");
    if (pr->levels == 2) {
        if (pb->stencil != ISDC_STENCIL_2ND || pb->bc != ISDC_BC_DIRICHLET)
            fail(ISDC_E_UNSUPPORTED, "two-level MLSDC runs the second-order stencil with Dirichlet boundaries");
        if (pb->n[0] < 3) fail(ISDC_E_INVAL, "two-level MLSDC needs n >= 3 to coarsen");
    }
    if (pb->bc == ISDC_BC_PERIODIC && pb->stencil != ISDC_STENCIL_COMPACT4)
        fail(ISDC_E_UNSUPPORTED, "periodic boundaries are implemented with the compact stencil only");
    if (pb->fe_kind == ISDC_FE_BURGERS && pb->bc != ISDC_BC_PERIODIC)
        fail(ISDC_E_UNSUPPORTED, "the WENO5 Burgers advection needs periodic boundaries");
}

namespace {
// Points per axis and spacing of multigrid level l (periodic: n -> n/2 on
// [-1, 1); Dirichlet: n -> (n-1)/2 interior points of (0, 1)).
void level_size(bool periodic, int n0, int l, int& n, double& h) {
    n = n0;
    h = periodic ? 2.0 / n0 : 1.0 / (n0 + 1);
    for (int i = 0; i < l; ++i) {
        n = periodic ? n / 2 : (n - 1) / 2;
        h *= 2.0;
    }
}
int level_count(bool periodic, int n0) {
    int nl = 1;
    for (int n = n0; n > 1; n = periodic ? n / 2 : (n - 1) / 2) ++nl;
    return nl;
}
}  // namespace

// Lay the plan's arrays out from `base` (nullptr: sizing only); returns the byte count.
size_t isdc::layout(const isdc_problem& pb, const isdc_params& pr, char* base, isdc_plan* p) {
    const int d = pb.dim, M = pr.M;
    const size_t N = pow_d((size_t)pb.n[0], d);
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* ptr = base ? (void*)(base + off) : nullptr;
        off = align_up(off + bytes);
        return ptr;
    };
    double tau[ISDC_MAX_M];
    tables(pr.node_kind, M, tau, nullptr, nullptr);
    for (int w = 0; w < 2; ++w)
        for (int j = 1; j <= M; ++j) {
            bool alias_u0 = (j == 1 && pr.node_kind == ISDC_NODES_LOBATTO);  // tau_1 = 0: u_1 = u_0
            void* ptr = alias_u0 ? nullptr : take(N * sizeof(double));
            if (p) p->U[w][j] = (double*)ptr;
        }
    for (int m = 0; m < M; ++m) {
        bool degenerate = (m == 0 && pr.node_kind == ISDC_NODES_LOBATTO);
        void* ptr = degenerate ? nullptr : take(N * sizeof(double));
        if (p) p->SF[m] = (double*)ptr;
    }
    const bool periodic = pb.bc == ISDC_BC_PERIODIC;
    if (pb.fe_kind == ISDC_FE_BURGERS) {  // f^E arrays beside u_0 and every node array
        void* f0 = take(N * sizeof(double));
        if (p) p->FE0 = (double*)f0;
        for (int w = 0; w < 2; ++w)
            for (int j = 1; j <= M; ++j) {
                bool alias_u0 = (j == 1 && pr.node_kind == ISDC_NODES_LOBATTO);
                void* ptr = alias_u0 ? nullptr : take(N * sizeof(double));
                if (p) p->FEU[w][j] = (double*)ptr;
            }
    }
    // multigrid hierarchy: 8 bytes per entry so either precision fits
    const int tmax = periodic ? kCTailMaxPeriodic : tail_max_n(d);
    int n = pb.n[0];
    double h = periodic ? 2.0 / pb.n[0] : 1.0 / (pb.n[0] + 1);
    int l = 0;
    if (p) p->lev.clear();
    while (true) {
        Level L{n, h, pow_d((size_t)n, d), nullptr, nullptr, nullptr};
        bool is_tail = n <= tmax;
        L.r = take(L.N * sizeof(double));
        L.e = take(L.N * sizeof(double));
        if (!is_tail || l == 0) L.e2 = take(L.N * sizeof(double));
        if (p) {
            p->lev.push_back(L);
            if (is_tail) p->tail = l;
        }
        if (is_tail) break;
        n = periodic ? n / 2 : (n - 1) / 2;
        h *= 2.0;
        ++l;
    }
    if (pr.levels == 2 && l == 0) {
        // the fine grid is small enough for the tail: the coarse MLSDC level
        // still needs arrays of its own, solved by the tail as well
        n = (n - 1) / 2;
        h *= 2.0;
        Level C{n, h, pow_d((size_t)n, d), nullptr, nullptr, nullptr};
        C.r = take(C.N * sizeof(double));
        C.e = take(C.N * sizeof(double));
        if (p) p->lev.push_back(C);
    }
    const bool compact = pb.stencil == ISDC_STENCIL_COMPACT4;
    if (compact)
        for (int m = 0; m < M; ++m) {
            bool zero_row = (m == 0 && pr.node_kind == ISDC_NODES_LOBATTO);  // Q row of tau_1 = 0
            void* y = zero_row ? nullptr : take(N * sizeof(double));
            void* x = zero_row ? nullptr : take(N * sizeof(double));
            if (p) {
                p->Yq[m] = (double*)y;
                p->X[m] = (double*)x;
            }
        }
    if (compact) {
        void* wx = take(N * sizeof(double));
        void* wd0 = take(N * sizeof(double));
        void* wd1 = take(N * sizeof(double));
        if (p) {
            p->WX = (double*)wx;
            p->WD[0] = (double*)wd0;
            p->WD[1] = (double*)wd1;
        }
    }
    size_t nparts = quad_partials(d, pb.n[0]) > kReduceBlocks ? quad_partials(d, pb.n[0]) : kReduceBlocks;
    if (compact) {
        const size_t rows = (size_t)pb.n[0] * ((pb.n[0] + 255) / 256);  // residual-norm blocks of the finest level
        nparts = std::max(nparts, std::max(rows, (size_t)kCResBlocks * M));
    }
    if (pr.levels == 2) {  // coarse MLSDC level: R U_j, the coarse sweep's values, injected S F
        const size_t Nc = pow_d((size_t)((pb.n[0] - 1) / 2), d);
        const bool lob = pr.node_kind == ISDC_NODES_LOBATTO;  // node 1 is u_0 on both levels
        for (int j = 0; j <= M; ++j) {
            void* r = (j == 1 && lob) ? nullptr : take(Nc * sizeof(double));
            void* u = (j == 0 || (j == 1 && lob)) ? nullptr : take(Nc * sizeof(double));
            if (p) {
                p->Rf[j] = r ? (double*)r : p->Rf[0];
                p->Uc[j] = u ? (double*)u : p->Rf[0];
            }
        }
        for (int m = 0; m < M; ++m) {
            void* sfc = (m == 0 && lob) ? nullptr : take(Nc * sizeof(double));
            if (p) p->SFc[m] = (double*)sfc;
        }
    }
    void* endq = pr.node_kind == ISDC_NODES_LEGENDRE ? take(N * sizeof(double)) : nullptr;
    if (p) p->END = (double*)endq;
    void* part = take(nparts * sizeof(double));
    void* sc = take(16 * sizeof(double));
    if (p) {
        p->partial = (double*)part;
        p->scalars = (double*)sc;
    }
    (void)tau;
    return off;
}

namespace {

void ensure_pinned(isdc_plan* p) {
    if (!p->h_pinned) {
        void* ptr = nullptr;
        HIPCHK(hipHostMalloc(&ptr, 64, hipHostMallocDefault));
        p->h_pinned = (double*)ptr;
    }
}

// Arms the plan's probe for the launch made in this scope if that launch is of
// the followed kind and level and its turn in the sample (isdc_probe_arm);
// `bytes` are its algorithmic bytes.  A probe the launcher did not consume
// (no launch was made) is handed back.
struct ProbeScope {
    isdc_plan* p;
    bool armed = false;
    ProbeScope(isdc_plan* plan, int kind, int level, double bytes) : p(plan) {
        ProbeState& pr = p->probe;
        if (pr.kind != kind || pr.level != level) return;
        if (pr.seen++ % pr.every != 0 || pr.used >= pr.limit) return;
        armed_probe() = &pr.pool[pr.used++];
        pr.bytes += bytes;
        armed = true;
        pending_bytes = bytes;
    }
    ~ProbeScope() {
        if (armed && armed_probe()) {  // not consumed
            armed_probe() = nullptr;
            p->probe.used -= 1;
            p->probe.bytes -= pending_bytes;
        }
    }
    double pending_bytes = 0.0;
};

// Algorithmic bytes of one launch of a followed multigrid kernel on level l
// (every array element read or written once; w = bytes per V-cycle value).
double mg_bytes(const isdc_plan* p, int kind, int l) {
    const double w = p->par.precision == ISDC_PREC_MIXED ? 4.0 : 8.0;
    const double N = (double)p->lev[l].N;
    const double Nc = l + 1 < (int)p->lev.size() ? (double)p->lev[l + 1].N : 0.0;
    switch (kind) {
        case ISDC_KERNEL_SMOOTH_RESTRICT: return (3.0 * N + Nc) * w;  // rhs, e in; e, coarse rhs out
        case ISDC_KERNEL_ZSMOOTH_RESTRICT: return (2.0 * N + Nc) * w; // rhs in; e, coarse rhs out
        case ISDC_KERNEL_SMOOTH: return 3.0 * N * w;                  // rhs, e in; e out
        case ISDC_KERNEL_RESTRICT: return (2.0 * N + Nc) * w;         // rhs, e in; coarse rhs out
        case ISDC_KERNEL_PROLONG_SMOOTH: return (3.0 * N + Nc) * w;   // rhs, e, coarse e in; e out
        case ISDC_KERNEL_PROLONG_UPDATE: return (2.0 * N + Nc) * w + 16.0 * N;  // + float64 g in, u out
        case ISDC_KERNEL_TAIL: return 2.0 * N * w;
        default: return 0.0;
    }
}

double read_scalar(isdc_plan* p, const double* d_src, hipStream_t s) {
    ensure_pinned(p);
    HIPCHK(hipMemcpyAsync(p->h_pinned, d_src, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return p->h_pinned[0];
}

// ---------------------------------------------------------------- V-cycle schedule

// Node update fused into the last kernel of a solve: u_out = g + e (mode 1)
// or u_out = e (mode 2, zero guess).  mode 0: no fusion.
struct Fuse {
    int mode = 0;
    const double* g = nullptr;
    double* u_out = nullptr;
};

template <typename T>
void smooth_steps(isdc_plan* p, const MGConfig& mg, int nsteps, int l, const Coef<T>& co, bool& zero, const T* rhs,
                  T*& cur, T*& other, hipStream_t s, int shape) {
    const int n = p->lev[l].n;
    for (int k = 0; k < nsteps; ++k) {
        if (mg.smoother == ISDC_SMOOTH_RBGS) {
            ProbeScope probe(p, zero ? -2 : ISDC_KERNEL_SMOOTH, l, mg_bytes(p, ISDC_KERNEL_SMOOTH, l));
            HIPCHK(launch_rbgs_tile<T>(p->d, n, co, zero, rhs, cur, other, s, shape));
        } else
            HIPCHK(launch_smooth<T>(mg, n, co, zero, rhs, cur, other, s));
        std::swap(cur, other);
        zero = false;
    }
}

// One V-cycle on a 2D Dirichlet level l with weighted-Jacobi smoothing of the
// second-order operator, on the fused row-tile kernels: the last (up to
// three) pre-smoothing steps with the residual's restriction in one launch,
// the prolongation with the first (up to three) post-smoothing steps in
// another; further steps three per launch.  Result in e (tmp: scratch of the
// level's size).
template <typename T>
bool jvcycle5_rec(isdc_plan* p, const MGConfig& mg, int l, double c, bool zero, const T* rhs, T* e, T* tmp,
                  hipStream_t s, const Fuse& fuse = Fuse()) {
    const Level& L = p->lev[l];
    if (l >= p->tail) {
        ProbeScope probe(p, l == p->tail ? ISDC_KERNEL_TAIL : -2, 0, mg_bytes(p, ISDC_KERNEL_TAIL, l));
        HIPCHK(launch_tail<T>(mg, L.n, c, L.h, zero, rhs, e, s));
        return false;
    }
    const CCoef<T> k = make_coef5<T>(c, L.h, mg.omega);
    T* cur = e;
    T* other = tmp;
    const Level& C = p->lev[l + 1];
    int pre = mg.nu_pre;
    while (pre > 3) {
        HIPCHK(launch_jacobi5_steps<T>(L.n, k, 3, zero, rhs, cur, other, s));
        std::swap(cur, other);
        zero = false;
        pre -= 3;
    }
    if (pre > 0) {
        ProbeScope probe(p, zero ? -2 : ISDC_KERNEL_SMOOTH_RESTRICT, l, mg_bytes(p, ISDC_KERNEL_SMOOTH_RESTRICT, l));
        HIPCHK(launch_jres5<T>(L.n, k, pre, zero, rhs, cur, other, (T*)C.r, s));
        std::swap(cur, other);
        zero = false;
    } else {
        if (zero) {
            HIPCHK(launch_fill<T>(cur, L.N, T(0), s));
            zero = false;
        }
        const Coef<T> co = make_coef<T>(c, L.h, p->d, mg.omega);
        HIPCHK(launch_restrict_tile<T>(p->d, L.n, co, rhs, cur, (T*)C.r, s));
    }
    jvcycle5_rec<T>(p, mg, l + 1, c, true, (const T*)C.r, (T*)C.e, (T*)C.e2, s);
    int post = mg.nu_post;
    if (post > 0) {
        const int first = std::min(3, post);
        // a single post-smoothing launch can write the node value g + e itself
        if (post == first && fuse.mode == 1) {
            ProbeScope probe(p, ISDC_KERNEL_PROLONG_UPDATE, l, mg_bytes(p, ISDC_KERNEL_PROLONG_UPDATE, l));
            HIPCHK(launch_pjac5<T>(L.n, k, first, rhs, cur, (const T*)C.e, other, fuse.g, fuse.u_out, s));
            return true;
        }
        {
            ProbeScope probe(p, ISDC_KERNEL_PROLONG_SMOOTH, l, mg_bytes(p, ISDC_KERNEL_PROLONG_SMOOTH, l));
            HIPCHK(launch_pjac5<T>(L.n, k, first, rhs, cur, (const T*)C.e, other, nullptr, nullptr, s));
        }
        std::swap(cur, other);
        post -= first;
        while (post > 0) {
            const int ks = std::min(3, post);
            HIPCHK(launch_jacobi5_steps<T>(L.n, k, ks, false, rhs, cur, other, s));
            std::swap(cur, other);
            post -= ks;
        }
    } else {
        HIPCHK(launch_prolong<T>(2, L.n, (const T*)C.e, cur, s));
    }
    if (cur != e) HIPCHK(launch_copy<T>(cur, e, L.N, s));
    return false;
}

// One V-cycle on level l for (I - c L) e = rhs starting from e (or from zero);
// the result ends in `e` (or, with fuse.mode != 0 on a fused path, goes to
// fuse.u_out and `e` is left unspecified).  tmp: a scratch array of the
// level's size.  Returns true if the fused update was done.
template <typename T>
bool vcycle_rec(isdc_plan* p, const MGConfig& mg, int l, double c, bool zero, const T* rhs, T* e, T* tmp, hipStream_t s,
                const Fuse& fuse = Fuse(), const RhsArgs* fra = nullptr) {
    const Level& L = p->lev[l];
    if (l >= p->tail) {  // (beyond the tail only the coarse MLSDC level, solved the same way)
        ProbeScope probe(p, l == p->tail ? ISDC_KERNEL_TAIL : -2, 0, mg_bytes(p, ISDC_KERNEL_TAIL, l));
        HIPCHK(launch_tail<T>(mg, L.n, c, L.h, zero, rhs, e, s));
        return false;
    }
    const bool rbgs = mg.smoother == ISDC_SMOOTH_RBGS;
    if (!rbgs && p->d == 2)  // 2D Jacobi: the fused row-tile kernels
        return jvcycle5_rec<T>(p, mg, l, c, zero, rhs, e, tmp, s, fuse);
    Coef<T> co = make_coef<T>(c, L.h, p->d, mg.omega);
    T* cur = e;
    T* other = tmp;
    const Level& C = p->lev[l + 1];
    if (rbgs && mg.nu_pre >= 1 && rbgs_restrict_fused(p->d, L.n)) {
        // pre-smoothing steps; the last one fused with residual + restriction
        smooth_steps<T>(p, mg, mg.nu_pre - 1, l, co, zero, rhs, cur, other, s, L.shape);
        if (fra && zero && mg.nu_pre == 1 && p->d == 2)  // rhs formed in the first launch (writes rhs)
            HIPCHK(launch_rhs_rbgs_restrict_tile<T>(p->d, L.n, *fra, co, (T*)rhs, other, (T*)C.r, s, L.shape));
        else {
            const int kind = zero ? ISDC_KERNEL_ZSMOOTH_RESTRICT : ISDC_KERNEL_SMOOTH_RESTRICT;
            ProbeScope probe(p, kind, l, mg_bytes(p, kind, l));
            HIPCHK(launch_rbgs_restrict_tile<T>(p->d, L.n, co, zero, rhs, cur, other, (T*)C.r, s, L.shape));
        }
        std::swap(cur, other);
        zero = false;
    } else {
        smooth_steps<T>(p, mg, mg.nu_pre, l, co, zero, rhs, cur, other, s, L.shape);
        if (zero) {  // no pre-smoothing and a zero iterate
            HIPCHK(launch_fill<T>(cur, L.N, T(0), s));
            zero = false;
        }
        ProbeScope probe(p, ISDC_KERNEL_RESTRICT, l, mg_bytes(p, ISDC_KERNEL_RESTRICT, l));
        HIPCHK(launch_restrict_tile<T>(p->d, L.n, co, rhs, cur, (T*)C.r, s));
    }
    vcycle_rec<T>(p, mg, l + 1, c, true, (const T*)C.r, (T*)C.e, (T*)C.e2, s);
    bool fused = false;
    if (rbgs && mg.nu_post >= 1) {
        // prolongation + correction fused with the first post-smoothing step
        const bool last = mg.nu_post == 1;
        const int mode = (last && fuse.mode) ? fuse.mode : 0;
        const int kind = mode == 0 ? ISDC_KERNEL_PROLONG_SMOOTH : (mode == 1 ? ISDC_KERNEL_PROLONG_UPDATE : -2);
        ProbeScope probe(p, kind, l, mg_bytes(p, kind, l));
        HIPCHK(launch_prolong_rbgs_tile<T>(p->d, L.n, co, rhs, cur, (const T*)C.e, other, fuse.g, fuse.u_out, mode, s,
                                           L.shape));
        if (mode) return true;
        std::swap(cur, other);
        smooth_steps<T>(p, mg, mg.nu_post - 1, l, co, zero, rhs, cur, other, s, L.shape);
    } else {
        HIPCHK(launch_prolong<T>(p->d, L.n, (const T*)C.e, cur, s));
        smooth_steps<T>(p, mg, mg.nu_post, l, co, zero, rhs, cur, other, s, L.shape);
    }
    if (cur != e) HIPCHK(launch_copy<T>(cur, e, L.N, s));
    return fused;
}

// The gate of a device-side stopping test is set for the launches of its scope.
struct GateScope {
    explicit GateScope(const int* g) { current_gate() = g; }
    ~GateScope() { current_gate() = nullptr; }
};

// Residual norm of level l followed by the device-side stopping test
// (launch_reduce_gate); both skip once the gate is set.
template <typename T>
void resnorm_gated(isdc_plan* p, int l, double c, const T* rhs, const T* u, double tol, int limit, int count_cycle,
                   int* gate, double* res_out, hipStream_t s) {
    const Level& L = p->lev[l];
    Coef<T> co = make_coef<T>(c, L.h, p->d, p->mg.omega);
    int nb = 0;
    HIPCHK(launch_resnorm<T>(p->d, L.n, co, rhs, u, p->partial, &nb, s));
    HIPCHK(launch_reduce_gate(p->partial, nb, tol, limit, count_cycle, gate, res_out, s));
}

template <typename T>
double resnorm(isdc_plan* p, int l, double c, const T* rhs, const T* u, hipStream_t s) {
    const Level& L = p->lev[l];
    Coef<T> co = make_coef<T>(c, L.h, p->d, p->mg.omega);
    int nb = 0;
    HIPCHK(launch_resnorm<T>(p->d, L.n, co, rhs, u, p->partial, &nb, s));
    HIPCHK(launch_reduce_max(p->partial, nb, p->scalars + 1, s));
    return read_scalar(p, p->scalars + 1, s);
}

// ---------------------------------------------------------------- SDC sweep

void quad_residual(isdc_plan* p, const double* const* nodes, hipStream_t s) {
    QuadArgs qa;
    std::memset(&qa, 0, sizeof(qa));
    for (int j = 0; j <= p->M; ++j) qa.u[j] = nodes[j];
    for (int m = 0; m < p->M; ++m) {
        qa.sf[m] = p->SF[m];
        for (int j = 0; j < p->M; ++j) {
            qa.dtS[m * ISDC_MAX_M + j] = p->dt * p->S[m * p->M + j];
            qa.dtQ[m * ISDC_MAX_M + j] = p->dt * p->Q[m * p->M + j];
        }
    }
    qa.nu_h2 = p->prob.nu / (p->h * p->h);
    qa.M = p->M;
    qa.n = p->n;
    qa.fe = p->prob.fe_kind;
    int nb = 0;
    {
        // algorithmic bytes: u_0 and every distinct node array read, the S F arrays written
        int arrays = 1;
        for (int j = 1; j <= p->M; ++j) arrays += nodes[j] != nodes[0];
        for (int m = 0; m < p->M; ++m) arrays += p->SF[m] != nullptr;
        ProbeScope probe(p, ISDC_KERNEL_QUAD, 0, (double)arrays * (double)p->N * 8.0);
        HIPCHK(launch_quad_residual(p->d, qa, p->partial, &nb, s));
    }
    HIPCHK(launch_reduce_max(p->partial, nb, p->scalars, s));
}

// ---------------------------------------------------------------- compact stencil (eq. (5))

// W^{-1} for the residual (Sec. 3): Chebyshev iteration on W = I + (h^2/12) L_h,
// whose Jacobi-scaled spectrum lies in [1/2, 3/2], so the error falls by at
// least (sqrt(3) - 1) / (sqrt(3) + 1) = 0.268 per step: 28 steps from zero
// (below 1e-15 relative) after the first sweep of a step, then 12 steps
// warm-started from the previous sweep's value (the change of W^{-1} Y between
// sweeps shrinks with the SDC residual).
constexpr int kWColdSteps = 28;
constexpr int kWWarmSteps = 12;

// One V-cycle of B_H = I + w L_H - c A_H with weighted-Jacobi smoothing on
// level l; same contract as vcycle_rec (result in e; tmp: scratch of the level).
template <typename T>
void cvcycle_rec(isdc_plan* p, const MGConfig& mg, int l, double c, bool zero, const T* rhs, T* e, T* tmp,
                 hipStream_t s) {
    const Level& L = p->lev[l];
    const bool per = p->periodic;
    if (l == p->tail) {
        HIPCHK(launch_ctail<T>(mg, L.n, c, p->w, L.h, zero, rhs, e, per, s));
        return;
    }
    const CCoef<T> k = make_ccoef<T>(c, p->w, L.h, mg.omega);
    T* cur = e;
    T* other = tmp;
    const Level& C = p->lev[l + 1];
    // pre-smoothing: the last (up to three) Jacobi steps fused with the
    // residual's restriction, earlier ones three per launch
    int pre = mg.nu_pre;
    while (pre > 3) {
        HIPCHK(launch_cjacobi_steps<T>(L.n, k, 3, zero, rhs, cur, other, per, s));
        std::swap(cur, other);
        zero = false;
        pre -= 3;
    }
    if (pre > 0) {
        HIPCHK(launch_cjres<T>(L.n, k, pre, zero, rhs, cur, other, (T*)C.r, per, s));
        std::swap(cur, other);
        zero = false;
    } else {
        if (zero) {
            HIPCHK(launch_fill<T>(cur, L.N, T(0), s));
            zero = false;
        }
        HIPCHK(launch_cresfw<T>(L.n, k, rhs, cur, (T*)C.r, per, s));
    }
    cvcycle_rec<T>(p, mg, l + 1, c, true, (const T*)C.r, (T*)C.e, (T*)C.e2, s);
    // post-smoothing: the prolongation fused with the first (up to three)
    // Jacobi steps, later ones three per launch
    int post = mg.nu_post;
    if (post > 0) {
        const int first = std::min(3, post);
        HIPCHK(launch_cpjac<T>(L.n, k, first, rhs, cur, (const T*)C.e, other, per, s));
        std::swap(cur, other);
        post -= first;
        while (post > 0) {
            const int ks = std::min(3, post);
            HIPCHK(launch_cjacobi_steps<T>(L.n, k, ks, false, rhs, cur, other, per, s));
            std::swap(cur, other);
            post -= ks;
        }
    } else if (per) {
        HIPCHK(launch_cprolong_p<T>(L.n, (const T*)C.e, cur, s));
    } else {
        HIPCHK(launch_prolong<T>(2, L.n, (const T*)C.e, cur, s));
    }
    if (cur != e) HIPCHK(launch_copy<T>(cur, e, L.N, s));
}

template <typename T>
double cresnorm(isdc_plan* p, int l, double c, const T* rhs, const T* u, hipStream_t s) {
    const Level& L = p->lev[l];
    int nb = 0;
    HIPCHK(launch_cresnorm<T>(L.n, make_ccoef<T>(c, p->w, L.h, p->mg.omega), rhs, u, p->partial, &nb, p->periodic, s));
    HIPCHK(launch_reduce_max(p->partial, nb, p->scalars + 1, s));
    return read_scalar(p, p->scalars + 1, s);
}

// The compact system of substep m in correction form (r in lev[0].r):
// L V-cycles from e = 0 (or cycles until the inner residual <= inner_tol),
// then u_out = g + e.
template <typename T>
int cinner_solve(isdc_plan* p, double c, const double* g, double* u_out, hipStream_t s) {
    const Level& L0 = p->lev[0];
    T* r0 = (T*)L0.r;
    T* e0 = (T*)L0.e;
    T* t0 = (T*)L0.e2;
    const isdc_params& pr = p->par;
    const bool classical = pr.vcycles == 0;
    const bool check = classical || pr.early_exit;
    const int limit = classical ? 100 : pr.vcycles;
    int k = 0;
    if (!check) {
        for (; k < limit; ++k) cvcycle_rec<T>(p, p->mg, 0, c, k == 0, r0, e0, t0, s);
    } else {
        HIPCHK(launch_fill<T>(e0, L0.N, T(0), s));
        for (; k < limit; ++k) {
            if (cresnorm<T>(p, 0, c, r0, e0, s) <= pr.inner_tol) break;
            cvcycle_rec<T>(p, p->mg, 0, c, false, r0, e0, t0, s);
        }
    }
    HIPCHK(launch_node_update<T>(p->N, ISDC_GUESS_PREV_SWEEP, g, g, e0, u_out, s));
    return k;
}

// S F~ for the next sweep and dt Q F~ for the residual from the node values
// (and their f^E arrays when f^E is a stencil).
void cquad(isdc_plan* p, const double* const* nodes, const double* const* fe, hipStream_t s) {
    CQuadArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int j = 0; j <= p->M; ++j) {
        a.u[j] = nodes[j];
        a.feu[j] = p->fe_arrays ? fe[j] : nullptr;
    }
    for (int m = 0; m < p->M; ++m) {
        a.sf[m] = p->SF[m];
        a.y[m] = p->Yq[m];
        for (int j = 0; j < p->M; ++j) {
            a.dtS[m * ISDC_MAX_M + j] = p->dt * p->S[m * p->M + j];
            a.dtQ[m * ISDC_MAX_M + j] = p->dt * p->Q[m * p->M + j];
        }
    }
    a.nu_6h2 = p->prob.nu / (6.0 * p->h * p->h);
    a.n = p->n;
    a.fe = p->prob.fe_kind;
    a.M = p->M;
    HIPCHK(launch_cquad(a, p->M, p->periodic, s));
}

// max over nodes and points of |u_0 + W^{-1} (dt Q F~)_m - u_m| (Sec. 3: W is
// inverted once per node), after cquad of the same node values.  W = I + w L:
// Dirichlet plans invert it with red-black V(1,1) cycles of the second-order
// solver (c = -w); periodic plans with the compact Jacobi cycle at c = 0.
// `steps` Chebyshev steps for W x = y from x = 0 (zero) or from x; tmp and d
// are scratch arrays of the finest level.  Even step counts end in x.
void wsolve(isdc_plan* p, bool zero, int steps, const double* y, double* x, hipStream_t s) {
    double* cur = x;
    double* other = p->WX;
    double* d = p->WD[0];
    double* d2 = p->WD[1];
    double rho = 0.5;  // 1 / sigma, sigma = centre / half-width = 2
    // the coefficients of every step, then launches of kWChebSteps fused steps
    // (single steps for a remainder)
    std::vector<double> cdv(steps, 0.0), crv(steps, 0.0);
    for (int k = 1; k < steps; ++k) {
        const double rn = 1.0 / (4.0 - rho);  // 1 / (2 sigma - rho)
        cdv[k] = rn * rho;
        crv[k] = 4.0 * rn;  // 2 rho_k / half-width
        rho = rn;
    }
    for (int k = 0; k < steps;) {
        const int kind = k == 0 ? (zero ? 0 : 1) : 2;
        if (steps - k >= kWChebSteps) {
            // the fused steps read d on a halo, so it is written out of place
            HIPCHK(launch_wcheb_steps(p->n, p->periodic, kind, kWChebSteps, y, cur, other, d, d2, &cdv[k], &crv[k],
                                      s));
            std::swap(d, d2);
            k += kWChebSteps;
        } else {
            HIPCHK(launch_wcheb(p->n, p->periodic, kind, y, cur, other, d, cdv[k], crv[k], s));
            ++k;
        }
        std::swap(cur, other);
    }
    if (cur != x) HIPCHK(launch_copy<double>(cur, x, p->N, s));
}

double cresidual(isdc_plan* p, hipStream_t s) {
    CResArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.u0 = p->u0;
    ra.N = p->N;
    const int steps = p->x_valid ? kWWarmSteps : kWColdSteps;
    for (int m = 0; m < p->M; ++m) {
        if (!p->Yq[m]) continue;
        wsolve(p, !p->x_valid, steps, p->Yq[m], p->X[m], s);
        ra.um[ra.count] = p->cur[m + 1];
        ra.xm[ra.count] = p->X[m];
        ++ra.count;
    }
    p->x_valid = true;
    int nb = 0;
    HIPCHK(launch_cres(ra, p->partial, &nb, s));
    HIPCHK(launch_reduce_max(p->partial, nb, p->scalars, s));
    return read_scalar(p, p->scalars, s);
}

// The implicit solve of substep m in correction form: the right-hand side
// r = rhs - A g is in lev[0].r; L V-cycles from e = 0 (or cycles until the
// inner residual <= inner_tol), then u_out = g + e.  The update is fused into
// the last V-cycle's final kernel when possible.
template <typename T>
int inner_solve(isdc_plan* p, double c, const Fuse& upd, hipStream_t s, const RhsArgs* fra = nullptr) {
    const Level& L0 = p->lev[0];
    T* r0 = (T*)L0.r;
    T* e0 = (T*)L0.e;
    T* t0 = (T*)L0.e2;
    const isdc_params& pr = p->par;
    const bool classical = pr.vcycles == 0;
    const bool check = classical || pr.early_exit;
    const int limit = classical ? 100 : pr.vcycles;
    int k = 0;
    bool fused = false;
    if (!check) {
        for (; k < limit; ++k)
            fused = vcycle_rec<T>(p, p->mg, 0, c, k == 0, r0, e0, t0, s, k == limit - 1 ? upd : Fuse(),
                                  k == 0 ? fra : nullptr);
    } else if (!p->compact) {
        // The stopping test runs on the device (k_reduce_gate): after the
        // first test the host enqueues a run of (cycle, test) pairs -- as many
        // as the same substep needed in its last solve -- and reads the gate
        // once; each test lets the next cycle run or stops the solve, and the
        // kernels of cycles after a stop return at once.  Only if the
        // tolerance is still unmet does another run follow.
        int* gate = (int*)(p->scalars + 8);
        double* res_out = p->scalars + 10;
        HIPCHK(launch_fill<T>(e0, L0.N, T(0), s));
        HIPCHK(launch_gate_reset(gate, s));
        {
            GateScope gs(gate);
            resnorm_gated<T>(p, 0, c, r0, e0, pr.inner_tol, limit, 1, gate, res_out, s);
        }
        int* hint = p->stats.sweeps == 0 ? p->gate_hint_first : p->gate_hint;
        int& h = hint[p->gate_substep];
        int run = std::max(1, std::min(h > 0 ? h : 3, limit));
        int enq = 0;  // cycles enqueued
        while (true) {
            {
                GateScope gs(gate);
                for (int q = 0; q < run && enq < limit; ++q, ++enq) {
                    vcycle_rec<T>(p, p->mg, 0, c, false, r0, e0, t0, s);
                    resnorm_gated<T>(p, 0, c, r0, e0, pr.inner_tol, limit, 1, gate, res_out, s);
                }
            }
            int g[2];
            HIPCHK(hipMemcpyAsync(g, gate, sizeof(g), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            k = g[1];
            if (g[0] || enq >= limit) break;
            run = 1;
        }
        h = k;
        p->gate_hint[p->gate_substep] = k;
    } else {
        HIPCHK(launch_fill<T>(e0, L0.N, T(0), s));
        for (; k < limit; ++k) {
            double res = resnorm<T>(p, 0, c, r0, e0, s);
            if (res <= pr.inner_tol) break;
            vcycle_rec<T>(p, p->mg, 0, c, false, r0, e0, t0, s);
        }
    }
    if (!fused) {
        if (k == 0 && !check) HIPCHK(launch_fill<T>(e0, L0.N, T(0), s));
        const int guess = upd.mode == 2 ? ISDC_GUESS_ZERO : ISDC_GUESS_PREV_SWEEP;
        HIPCHK(launch_node_update<T>(p->N, guess, upd.g, upd.g, e0, upd.u_out, s));
    }
    return k;
}

// True if a substep's right-hand side can be formed in the first launch of its
// solve (launch_rhs_rbgs_restrict_tile): 2D red-black V(1,1)-type cycles with
// one pre-smoothing step, a fixed number of cycles from e = 0 and the
// previous-sweep guess, for which the rhs is pointwise.
bool rhs_fusable(const isdc_plan* p) {
    return p->d == 2 && !p->compact && !p->periodic && p->par.guess == ISDC_GUESS_PREV_SWEEP &&
           p->mg.smoother == ISDC_SMOOTH_RBGS && p->mg.nu_pre == 1 && p->par.vcycles >= 1 && !p->par.early_exit &&
           p->tail >= 1 && (p->prob.fe_kind == ISDC_FE_ZERO || p->prob.fe_kind == ISDC_FE_CUBIC);
}

// The node loop of one sweep (eq. (4) / eq. (5)); afterwards cur[] holds the
// new iterate.  The quadrature of the new values is left to the caller.
template <typename T>
void sweep_nodes(isdc_plan* p, hipStream_t s) {
    const int M = p->M;
    double* const* W = p->U[p->wbuf];
    const double* nw[ISDC_MAX_M + 1];
    const double* nfe[ISDC_MAX_M + 1];  // f^E(nw[j]) (fe_arrays only)
    nw[0] = p->u0;
    nfe[0] = p->FE0;
    for (int j = 1; j <= M; ++j) {
        nw[j] = W[j] ? W[j] : p->u0;  // Lobatto node 1 is u_0
        nfe[j] = W[j] ? p->FEU[p->wbuf][j] : p->FE0;
    }
    const double nu_h2 = p->prob.nu / (p->h * p->h);
    for (int m = 0; m < M; ++m) {
        if (p->dtau[m] == 0.0) continue;  // tau_1 = 0 (Lobatto): u_1 = u_0, no solve
        const double dtm = p->dt * p->dtau[m];
        if (p->compact) {  // eq. (5)
            CRhsArgs ca{nw[m], p->cur[m], p->cur[m + 1], p->SF[m], dtm, p->n, p->prob.fe_kind, nullptr, nullptr};
            if (p->fe_arrays) {
                ca.fe_new = nfe[m];
                ca.fe_old = p->curfe[m];
            }
            HIPCHK(launch_crhs<T>(ca, (T*)p->lev[0].r, p->periodic, s));
            p->stats.vcycles += cinner_solve<T>(p, dtm * p->prob.nu, p->cur[m + 1], (double*)nw[m + 1], s);
            if (p->fe_arrays) HIPCHK(launch_weno_burgers(p->n, p->h, nw[m + 1], (double*)nfe[m + 1], s));
            continue;
        }
        RhsArgs ra{nw[m], p->cur[m], p->cur[m + 1], p->SF[m], dtm, dtm * p->prob.nu, nu_h2, p->n,
                   p->prob.fe_kind, p->par.guess};
        const bool fuse_rhs = rhs_fusable(p);
        if (!fuse_rhs) {
            // f^E = 0 reads u_m^{k+1}, u_{m+1}^k and S F; f^E != 0 also u_m^k (previous-sweep guess)
            const double reads = p->prob.fe_kind == ISDC_FE_ZERO ? 3.0 : 4.0;
            const double w = p->par.precision == ISDC_PREC_MIXED ? 4.0 : 8.0;
            ProbeScope probe(p, p->par.guess == ISDC_GUESS_PREV_SWEEP ? ISDC_KERNEL_RHS : -2, 0,
                             (reads * 8.0 + w) * (double)p->N);
            HIPCHK(launch_euler_rhs<T>(p->d, ra, (T*)p->lev[0].r, s));
        }
        Fuse upd;
        upd.u_out = (double*)nw[m + 1];
        if (p->par.guess == ISDC_GUESS_ZERO) {
            upd.mode = 2;
        } else {
            upd.mode = 1;
            upd.g = p->par.guess == ISDC_GUESS_PREV_NODE ? nw[m] : p->cur[m + 1];
        }
        p->gate_substep = m;
        p->stats.vcycles += inner_solve<T>(p, dtm * p->prob.nu, upd, s, fuse_rhs ? &ra : nullptr);
    }
    for (int j = 0; j <= M; ++j) {
        p->cur[j] = nw[j];
        p->curfe[j] = nfe[j];
    }
    p->wbuf ^= 1;
}

// The implicit solve of one coarse MLSDC substep: r in lev[1].r, the
// correction in lev[1].e; same modes as inner_solve.
template <typename T>
int coarse_solve(isdc_plan* p, double c, hipStream_t s) {
    const Level& L1 = p->lev[1];
    T* r1 = (T*)L1.r;
    T* e1 = (T*)L1.e;
    T* t1 = (T*)L1.e2;  // unused when level 1 is the single-workgroup tail
    const isdc_params& pr = p->par;
    const bool classical = pr.vcycles == 0;
    const bool check = classical || pr.early_exit;
    const int limit = classical ? 100 : pr.vcycles;
    int k = 0;
    if (!check) {
        for (; k < limit; ++k) vcycle_rec<T>(p, p->mg, 1, c, k == 0, r1, e1, t1, s);
        if (k == 0) HIPCHK(launch_fill<T>(e1, L1.N, T(0), s));
    } else {
        HIPCHK(launch_fill<T>(e1, L1.N, T(0), s));
        for (; k < limit; ++k) {
            if (resnorm<T>(p, 1, c, r1, e1, s) <= pr.inner_tol) break;
            vcycle_rec<T>(p, p->mg, 1, c, false, r1, e1, t1, s);
        }
    }
    return k;
}

// One two-level MLSDC iteration (Sec. 5): the fine sweep, injection of the
// node values and of S F to the (n-1)/2 grid, one coarse sweep, the coarse
// correction added back by cubic interpolation.  The coarse sweep's FAS term
// is not formed on its own: with tau_m = R(dt Q_m F_h) - dt Q_m F_2h(R U) the
// node-to-node sum of the coarse sweep, S_m F_2h(R U) + tau_{m+1} - tau_m,
// equals R(S_m F_h) exactly, and that is what the fine quadrature already
// wrote; the sweep's other terms use coarse values and the coarse operator.
template <typename T>
void mlsdc_iteration(isdc_plan* p, hipStream_t s) {
    const int M = p->M, d = p->d, n = p->n;
    sweep_nodes<T>(p, s);
    quad_residual(p, p->cur, s);  // S F of the new fine iterate (its residual is not used)
    for (int j = 0; j <= M; ++j)
        if (j == 0 || p->Rf[j] != p->Rf[0]) HIPCHK(launch_inject(d, n, p->cur[j], p->Rf[j], s));
    for (int m = 0; m < M; ++m)
        if (p->SFc[m]) HIPCHK(launch_inject(d, n, p->SF[m], p->SFc[m], s));
    const Level& L1 = p->lev[1];
    const double nu_h2c = p->prob.nu / (L1.h * L1.h);
    for (int m = 0; m < M; ++m) {
        if (p->dtau[m] == 0.0) continue;  // Lobatto: coarse node 1 is R u_0
        const double dtm = p->dt * p->dtau[m];
        const double* um_new = m == 0 ? p->Rf[0] : p->Uc[m];
        RhsArgs ra{um_new, p->Rf[m], p->Rf[m + 1], p->SFc[m], dtm, dtm * p->prob.nu, nu_h2c, L1.n,
                   p->prob.fe_kind, ISDC_GUESS_PREV_SWEEP};
        HIPCHK(launch_euler_rhs<T>(d, ra, (T*)L1.r, s));
        p->stats.coarse_vcycles += coarse_solve<T>(p, dtm * p->prob.nu, s);
        HIPCHK(launch_node_update<T>(L1.N, ISDC_GUESS_PREV_SWEEP, p->Rf[m + 1], p->Rf[m + 1], (const T*)L1.e,
                                     p->Uc[m + 1], s));
    }
    for (int j = 1; j <= M; ++j)
        if (p->cur[j] != p->u0) HIPCHK(launch_cubic_correct(d, n, p->Uc[j], p->Rf[j], (double*)p->cur[j], s));
}

template <typename T>
double sweep_impl(isdc_plan* p, hipStream_t s) {
    if (p->levels == 2)
        mlsdc_iteration<T>(p, s);
    else
        sweep_nodes<T>(p, s);
    double res;
    if (p->compact) {
        cquad(p, p->cur, p->curfe, s);
        res = cresidual(p, s);
    } else {
        quad_residual(p, p->cur, s);
        res = read_scalar(p, p->scalars, s);
    }
    p->stats.sweeps += 1;
    p->stats.residual = res;
    if (p->stats.hist_len < ISDC_HIST) p->stats.residual_hist[p->stats.hist_len++] = res;
    return res;
}

void begin_impl(isdc_plan* p, const double* d_u0, double dt, hipStream_t s) {
    if (!d_u0) fail(ISDC_E_INVAL, "d_u0 is NULL");
    if (!std::isfinite(dt) || dt <= 0) fail(ISDC_E_INVAL, "dt must be finite and > 0");
    p->u0 = d_u0;
    p->dt = dt;
    for (int j = 0; j <= p->M; ++j) p->cur[j] = d_u0;  // spread u_0 to every node
    p->wbuf = 0;
    p->begun = true;
    std::memset(&p->stats, 0, sizeof(p->stats));
    if (p->fe_arrays) {
        HIPCHK(launch_weno_burgers(p->n, p->h, d_u0, p->FE0, s));
        for (int j = 0; j <= p->M; ++j) p->curfe[j] = p->FE0;
    }
    if (p->compact) {
        cquad(p, p->cur, p->curfe, s);  // S*F~(u^0) for sweep 1
        p->x_valid = false;
    } else {
        quad_residual(p, p->cur, s);  // S*F(u^0) for sweep 1
    }
}

double sweep_any(isdc_plan* p, hipStream_t s) {
    if (!p->begun) fail(ISDC_E_INVAL, "isdc_sweep before isdc_begin");
    return p->par.precision == ISDC_PREC_MIXED ? sweep_impl<float>(p, s) : sweep_impl<double>(p, s);
}

// Gauss-Legendre steps end between the last node and T_{n+1}: the result is
// u_0 + dt sum_j b_j f(u_j) (Sec. 1), formed by the quadrature kernel with the
// weights b as its only row; the compact stencil keeps W f~, so W^{-1} is
// applied first (cold W steps, as for the residual of a step's first sweep).
void end_quadrature(isdc_plan* p, double* d_out, hipStream_t s) {
    const double* add = p->END;
    if (p->compact) {
        CQuadArgs a;
        std::memset(&a, 0, sizeof(a));
        for (int j = 0; j <= p->M; ++j) {
            a.u[j] = p->cur[j];
            a.feu[j] = p->fe_arrays ? p->curfe[j] : nullptr;
        }
        a.sf[0] = p->END;
        for (int j = 0; j < p->M; ++j) a.dtS[j] = p->dt * p->b[j];
        a.nu_6h2 = p->prob.nu / (6.0 * p->h * p->h);
        a.n = p->n;
        a.fe = p->prob.fe_kind;
        a.M = p->M;
        HIPCHK(launch_cquad(a, p->M, p->periodic, s));
        double* x = (double*)p->lev[0].e;
        wsolve(p, true, kWColdSteps, p->END, x, s);
        add = x;
    } else {
        QuadArgs qa;
        std::memset(&qa, 0, sizeof(qa));
        for (int j = 0; j <= p->M; ++j) qa.u[j] = p->cur[j];
        qa.sf[0] = p->END;
        for (int j = 0; j < p->M; ++j) qa.dtS[j] = p->dt * p->b[j];
        qa.nu_h2 = p->prob.nu / (p->h * p->h);
        qa.M = p->M;
        qa.n = p->n;
        qa.fe = p->prob.fe_kind;
        int nb = 0;  // the kernel's residual output is not used here
        HIPCHK(launch_quad_residual(p->d, qa, p->partial, &nb, s));
    }
    HIPCHK(launch_node_update<double>(p->N, ISDC_GUESS_PREV_SWEEP, p->u0, p->u0, add, d_out, s));
}

void end_impl(isdc_plan* p, double* d_out, hipStream_t s) {
    if (!p->begun) fail(ISDC_E_INVAL, "isdc_end before isdc_begin");
    if (!d_out) fail(ISDC_E_INVAL, "d_u_out is NULL");
    if (p->end_quad) {
        end_quadrature(p, d_out, s);
    } else {
        const double* src = p->cur[p->M];
        if (src != d_out) HIPCHK(hipMemcpyAsync(d_out, src, p->N * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    p->begun = false;
}

void check_plan(const isdc_plan* p) {
    if (!p) fail(ISDC_E_INVAL, "plan is NULL");
}

// One time step (Sec. 2-3): sweeps until the SDC residual is below sdc_tol,
// it is not finite, or max_sweeps is reached; returns the step's status.
int step_loop(isdc_plan* plan, double* d_u, double dt, hipStream_t s, isdc_stats* out) {
    if (!d_u) fail(ISDC_E_INVAL, "d_u is NULL");
    FILE* trace = trace_stream();
    const auto t0 = std::chrono::steady_clock::now();
    begin_impl(plan, d_u, dt, s);
    int status = ISDC_E_NOT_CONVERGED;
    for (int k = 0; k < plan->par.max_sweeps; ++k) {
        double res = sweep_any(plan, s);
        if (trace) {  // host time once the sweep's residual has been read back
            const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
            std::fprintf(trace, "isdc_trace plan=%p dim=%d n=%d sweep=%d t_us=%.1f residual=%.6e vcycles=%lld\n",
                         (void*)plan, plan->d, plan->n, k + 1, us, res, (long long)plan->stats.vcycles);
            std::fflush(trace);
        }
        if (!std::isfinite(res)) {
            status = ISDC_E_DIVERGED;
            break;
        }
        if (res < plan->par.sdc_tol) {
            status = ISDC_OK;
            break;
        }
    }
    end_impl(plan, d_u, s);
    if (out) *out = plan->stats;
    return status;
}

int step_status(const isdc_plan* plan, int status) {
    if (status == ISDC_E_NOT_CONVERGED)
        isdc::last_error() = "SDC residual " + std::to_string(plan->stats.residual) + " not below sdc_tol after max_sweeps";
    else if (status == ISDC_E_DIVERGED)
        isdc::last_error() = "non-finite SDC residual";
    return status;
}

// ---------------------------------------------------------------- static scratch
// isdc_step_noalloc lays its plan out on this device array instead of a caller
// workspace.  In host code `scratch` only names the symbol: its device address
// comes from hipGetSymbolAddress, once per device, and only that address is
// passed on.  Every device the library runs on holds its own copy until the
// process ends.
constexpr size_t kScratchBytes = ISDC_STATIC_SCRATCH_BYTES;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct StaticDevice {
    std::once_flag once;
    hipError_t err = hipSuccess;
    void* scratch_ptr = nullptr;  // this device's address of `scratch`
    isdc_plan* plan = nullptr;    // host plan shared by the calls on this device
    double readback[8];           // residual read-back target (ordinary host memory)
};
StaticDevice g_static[kMaxDevices];

// Set-up on the first call on the current device: the scratch address and a
// host plan whose level table is reserved and whose read-back target is the
// static host buffer, so later calls allocate nothing on the device or pinned.
StaticDevice& static_device() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(ISDC_E_UNSUPPORTED, "device index beyond the static scratch table");
    StaticDevice& sd = g_static[dev];
    std::call_once(sd.once, [&sd] {
        void* ptr = nullptr;
        sd.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (sd.err != hipSuccess) return;
        sd.scratch_ptr = ptr;
        sd.plan = new isdc_plan();
        sd.plan->lev.reserve(32);
        sd.plan->h_pinned = sd.readback;
    });
    if (sd.err != hipSuccess)
        fail(ISDC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(sd.err));
    return sd;
}

}  // namespace


void isdc::init_plan(isdc_plan* p, const isdc_problem* prob, const isdc_params* par, void* d_workspace) {
    p->prob = *prob;
    p->par = *par;
    p->d = prob->dim;
    p->n = prob->n[0];
    p->N = pow_d((size_t)prob->n[0], prob->dim);
    p->periodic = prob->bc == ISDC_BC_PERIODIC;
    p->h = p->periodic ? 2.0 / prob->n[0] : 1.0 / (prob->n[0] + 1);
    p->M = par->M;
    tables(par->node_kind, par->M, p->tau, p->Q, p->S, p->b);
    p->end_quad = par->node_kind == ISDC_NODES_LEGENDRE;
    p->levels = par->levels;
    std::memset(p->Rf, 0, sizeof(p->Rf));
    std::memset(p->Uc, 0, sizeof(p->Uc));
    std::memset(p->SFc, 0, sizeof(p->SFc));
    double prev = 0.0;
    for (int m = 0; m < p->M; ++m) {
        p->dtau[m] = p->tau[m] - prev;
        prev = p->tau[m];
    }
    p->compact = prob->stencil == ISDC_STENCIL_COMPACT4;
    p->w = p->h * p->h / 12.0;
    p->mg = MGConfig{p->d, par->smoother, par->nu_pre, par->nu_post,
                     p->compact ? 1.0 : 2.0 * p->d / (2.0 * p->d + 1.0)};
    p->fe_arrays = prob->fe_kind == ISDC_FE_BURGERS;
    p->FE0 = nullptr;
    std::memset(p->FEU, 0, sizeof(p->FEU));
    std::memset(p->curfe, 0, sizeof(p->curfe));
    p->x_valid = false;
    std::memset(p->Yq, 0, sizeof(p->Yq));
    std::memset(p->X, 0, sizeof(p->X));
    std::memset(p->U, 0, sizeof(p->U));
    std::memset(p->SF, 0, sizeof(p->SF));
    layout(*prob, *par, (char*)d_workspace, p);
    std::memset(&p->stats, 0, sizeof(p->stats));
    std::memset(p->gate_hint, 0, sizeof(p->gate_hint));
    std::memset(p->gate_hint_first, 0, sizeof(p->gate_hint_first));
    p->gate_substep = 0;
}

// ================================================================ C ABI

extern "C" {

int isdc_version(void) { return 100; }

int isdc_abi_sizes(size_t* problem, size_t* params, size_t* stats) {
    if (problem) *problem = sizeof(isdc_problem);
    if (params) *params = sizeof(isdc_params);
    if (stats) *stats = sizeof(isdc_stats);
    return ISDC_OK;
}

const char* isdc_last_error(void) { return isdc::last_error().c_str(); }

int isdc_default_params(isdc_params* p) {
    return guarded([&] {
        if (!p) fail(ISDC_E_INVAL, "params is NULL");
        p->node_kind = ISDC_NODES_LOBATTO;
        p->M = 3;
        p->vcycles = 2;
        p->inner_tol = 1e-10;
        p->early_exit = 0;
        p->sdc_tol = 1e-10;
        p->max_sweeps = 100;
        p->smoother = ISDC_SMOOTH_RBGS;
        p->nu_pre = 1;
        p->nu_post = 1;
        p->precision = ISDC_PREC_FP64;
        p->guess = ISDC_GUESS_PREV_SWEEP;
        p->levels = 1;
    });
}

int isdc_tables(int32_t node_kind, int32_t M, double* h_tau, double* h_Q, double* h_S) {
    return guarded([&] {
        if (!tables(node_kind, M, h_tau, h_Q, h_S)) fail(ISDC_E_INVAL, "invalid node_kind or M");
    });
}

int isdc_end_weights(int32_t node_kind, int32_t M, double* h_b) {
    return guarded([&] {
        if (!h_b) fail(ISDC_E_INVAL, "h_b is NULL");
        if (!tables(node_kind, M, nullptr, nullptr, nullptr, h_b)) fail(ISDC_E_INVAL, "invalid node_kind or M");
    });
}

int isdc_workspace_bytes(const isdc_problem* prob, const isdc_params* par, size_t* out_bytes) {
    return guarded([&] {
        validate(prob, par);
        if (!out_bytes) fail(ISDC_E_INVAL, "out_bytes is NULL");
        *out_bytes = layout(*prob, *par, nullptr, nullptr);
    });
}

int isdc_create(const isdc_problem* prob, const isdc_params* par, void* d_workspace, size_t bytes,
                isdc_plan** out_plan) {
    return guarded([&] {
        validate(prob, par);
        if (!out_plan) fail(ISDC_E_INVAL, "out_plan is NULL");
        *out_plan = nullptr;
        size_t need = layout(*prob, *par, nullptr, nullptr);
        if (!d_workspace) fail(ISDC_E_WORKSPACE, "workspace is NULL");
        if (((uintptr_t)d_workspace) % kAlign) fail(ISDC_E_WORKSPACE, "workspace must be 256-byte aligned");
        if (bytes < need) fail(ISDC_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
        isdc_plan* p = new isdc_plan();
        init_plan(p, prob, par, d_workspace);
        *out_plan = p;
    });
}

void isdc_destroy(isdc_plan* plan) {
    if (!plan) return;
    if (plan->h_pinned) (void)hipHostFree(plan->h_pinned);
    for (auto& ev : plan->probe.pool) {
        (void)hipEventDestroy(ev.start);
        (void)hipEventDestroy(ev.stop);
    }
    delete plan;
}

int isdc_probe_arm(isdc_plan* plan, int32_t kernel, int32_t level, int32_t every, int32_t max_samples) {
    return guarded([&] {
        check_plan(plan);
        if (plan->compact) fail(ISDC_E_UNSUPPORTED, "probes follow second-order stencil plans");
        const bool leveled = kernel == ISDC_KERNEL_SMOOTH_RESTRICT || kernel == ISDC_KERNEL_SMOOTH ||
                             kernel == ISDC_KERNEL_RESTRICT || kernel == ISDC_KERNEL_PROLONG_SMOOTH ||
                             kernel == ISDC_KERNEL_ZSMOOTH_RESTRICT;
        if (!leveled && kernel != ISDC_KERNEL_PROLONG_UPDATE && kernel != ISDC_KERNEL_TAIL &&
            kernel != ISDC_KERNEL_QUAD && kernel != ISDC_KERNEL_RHS)
            fail(ISDC_E_INVAL, "kernel cannot be followed by a probe");
        if (leveled && (level < 0 || level >= plan->tail)) fail(ISDC_E_INVAL, "level must lie above the coarse tail");
        if (every < 1 || every > 1000000) fail(ISDC_E_INVAL, "every must be in 1..1000000");
        if (max_samples < 1 || max_samples > 1000000) fail(ISDC_E_INVAL, "max_samples must be in 1..1000000");
        ProbeState& pr = plan->probe;
        while (pr.pool.size() < (size_t)max_samples) {
            LaunchProbe ev{};
            HIPCHK(hipEventCreate(&ev.start));
            HIPCHK(hipEventCreate(&ev.stop));
            pr.pool.push_back(ev);
        }
        pr.kind = kernel;
        pr.level = leveled ? level : 0;
        pr.every = every;
        pr.seen = 0;
        pr.used = 0;
        pr.bytes = 0.0;
        pr.limit = (size_t)max_samples;  // samples beyond max_samples are not taken
    });
}

int isdc_probe_read(isdc_plan* plan, int64_t* h_samples, double* h_avg_us, double* h_bytes) {
    return guarded([&] {
        check_plan(plan);
        ProbeState& pr = plan->probe;
        if (pr.kind < 0) fail(ISDC_E_INVAL, "no probe armed");
        double total_ms = 0.0;
        for (size_t k = 0; k < pr.used; ++k) {
            HIPCHK(hipEventSynchronize(pr.pool[k].stop));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, pr.pool[k].start, pr.pool[k].stop));
            total_ms += ms;
        }
        if (h_samples) *h_samples = (int64_t)pr.used;
        if (h_avg_us) *h_avg_us = pr.used ? 1e3 * total_ms / (double)pr.used : 0.0;
        if (h_bytes) *h_bytes = pr.used ? pr.bytes / (double)pr.used : 0.0;
        pr.kind = -1;
    });
}

int isdc_begin(isdc_plan* plan, const double* d_u0, double dt, void* stream) {
    return guarded([&] {
        check_plan(plan);
        begin_impl(plan, d_u0, dt, (hipStream_t)stream);
    });
}

int isdc_sweep(isdc_plan* plan, void* stream, double* h_residual) {
    return guarded([&] {
        check_plan(plan);
        double r = sweep_any(plan, (hipStream_t)stream);
        if (h_residual) *h_residual = r;
    });
}

int isdc_end(isdc_plan* plan, double* d_u_out, void* stream) {
    return guarded([&] {
        check_plan(plan);
        end_impl(plan, d_u_out, (hipStream_t)stream);
    });
}

int isdc_step(isdc_plan* plan, double* d_u, double dt, void* stream, isdc_stats* out) {
    int status = ISDC_OK;
    int rc = guarded([&] {
        check_plan(plan);
        status = step_loop(plan, d_u, dt, (hipStream_t)stream, out);
    });
    return rc != ISDC_OK ? rc : step_status(plan, status);
}

int isdc_step_noalloc(const isdc_problem* prob, const isdc_params* par, double* d_u, double dt, void* stream,
                      isdc_stats* out) {
    int status = ISDC_OK;
    isdc_plan* plan = nullptr;
    int rc = guarded([&] {
        validate(prob, par);
        const size_t need = layout(*prob, *par, nullptr, nullptr);
        if (need > kScratchBytes)
            fail(ISDC_E_WORKSPACE, "problem needs " + std::to_string(need) + " bytes of workspace; the static scratch holds " +
                                       std::to_string(kScratchBytes));
        if (!d_u) fail(ISDC_E_INVAL, "d_u is NULL");
        StaticDevice& sd = static_device();
        plan = sd.plan;
        init_plan(plan, prob, par, sd.scratch_ptr);
        status = step_loop(plan, d_u, dt, (hipStream_t)stream, out);
    });
    return rc != ISDC_OK ? rc : step_status(plan, status);
}

int isdc_node_values(isdc_plan* plan, int32_t j, double* d_out, void* stream) {
    return guarded([&] {
        check_plan(plan);
        if (!plan->begun) fail(ISDC_E_INVAL, "no step in progress (call isdc_begin first)");
        if (j < 0 || j > plan->M) fail(ISDC_E_INVAL, "node index out of range");
        if (!d_out) fail(ISDC_E_INVAL, "d_out is NULL");
        HIPCHK(hipMemcpyAsync(d_out, plan->cur[j], plan->N * sizeof(double), hipMemcpyDeviceToDevice,
                              (hipStream_t)stream));
    });
}

int isdc_get_stats(const isdc_plan* plan, isdc_stats* out) {
    return guarded([&] {
        check_plan(plan);
        if (!out) fail(ISDC_E_INVAL, "out is NULL");
        *out = plan->stats;
    });
}

int isdc_vcycle(isdc_plan* plan, double c, int32_t precision, const void* d_rhs, void* d_u, int32_t ncycles,
                void* stream, double* h_res_inf) {
    return guarded([&] {
        check_plan(plan);
        if (!std::isfinite(c) || c < 0) fail(ISDC_E_INVAL, "c must be finite and >= 0");
        if (precision != ISDC_PREC_FP64 && precision != ISDC_PREC_MIXED) fail(ISDC_E_INVAL, "unknown precision");
        if (!d_rhs || !d_u) fail(ISDC_E_INVAL, "NULL rhs or u");
        if (ncycles < 0) fail(ISDC_E_INVAL, "ncycles must be >= 0");
        hipStream_t s = (hipStream_t)stream;
        if (plan->compact) {
            if (precision == ISDC_PREC_FP64) {
                for (int k = 0; k < ncycles; ++k)
                    cvcycle_rec<double>(plan, plan->mg, 0, c, false, (const double*)d_rhs, (double*)d_u,
                                        (double*)plan->lev[0].e2, s);
                if (h_res_inf) *h_res_inf = cresnorm<double>(plan, 0, c, (const double*)d_rhs, (const double*)d_u, s);
            } else {
                for (int k = 0; k < ncycles; ++k)
                    cvcycle_rec<float>(plan, plan->mg, 0, c, false, (const float*)d_rhs, (float*)d_u,
                                       (float*)plan->lev[0].e2, s);
                if (h_res_inf) *h_res_inf = cresnorm<float>(plan, 0, c, (const float*)d_rhs, (const float*)d_u, s);
            }
            return;
        }
        if (precision == ISDC_PREC_FP64) {
            for (int k = 0; k < ncycles; ++k)
                vcycle_rec<double>(plan, plan->mg, 0, c, false, (const double*)d_rhs, (double*)d_u, (double*)plan->lev[0].e2, s);
            if (h_res_inf) *h_res_inf = resnorm<double>(plan, 0, c, (const double*)d_rhs, (const double*)d_u, s);
        } else {
            for (int k = 0; k < ncycles; ++k)
                vcycle_rec<float>(plan, plan->mg, 0, c, false, (const float*)d_rhs, (float*)d_u, (float*)plan->lev[0].e2, s);
            if (h_res_inf) *h_res_inf = resnorm<float>(plan, 0, c, (const float*)d_rhs, (const float*)d_u, s);
        }
    });
}

}  // extern "C"

namespace {

template <typename T>
void mg_op_impl(isdc_plan* p, int op, int level, double c, const void* a, const void* b, void* out, hipStream_t s,
                double* h_scalar) {
    const int d = p->d;
    if (op == ISDC_OP_EXPLICIT) {
        if (!p->fe_arrays) fail(ISDC_E_UNSUPPORTED, "EXPLICIT probes the WENO5 Burgers advection only");
        if (level != 0) fail(ISDC_E_INVAL, "EXPLICIT acts on the finest level");
        if (!a || !out) fail(ISDC_E_INVAL, "EXPLICIT needs input and output");
        if (a == out) fail(ISDC_E_INVAL, "EXPLICIT needs a separate output array");
        HIPCHK(launch_weno_burgers(p->n, p->h, (const double*)a, (double*)out, s));
        return;
    }
    int n;
    double h;
    level_size(p->periodic, p->n, level, n, h);
    const size_t N = pow_d((size_t)n, d);
    Coef<T> co = make_coef<T>(c, h, d, p->mg.omega);
    if (p->compact) {
        const bool per = p->periodic;
        const int nmin = per ? 2 : 3;
        const CCoef<T> k = make_ccoef<T>(c, p->w, h, p->mg.omega);
        switch (op) {
            case ISDC_OP_SMOOTH:
                if (!a || !b || !out) fail(ISDC_E_INVAL, "SMOOTH needs rhs, iterate and output");
                if (out == b) fail(ISDC_E_INVAL, "Jacobi SMOOTH needs a separate output array");
                HIPCHK(launch_cjacobi<T>(n, k, false, (const T*)a, (const T*)b, (T*)out, per, s));
                break;
            case ISDC_OP_RESTRICT:
                if (n < nmin) fail(ISDC_E_INVAL, "RESTRICT needs a level with a coarser level below it");
                if (!a || !b || !out) fail(ISDC_E_INVAL, "RESTRICT needs rhs, iterate and output");
                HIPCHK(launch_cresfw<T>(n, k, (const T*)a, (const T*)b, (T*)out, per, s));
                break;
            case ISDC_OP_PROLONG:
                if (n < nmin) fail(ISDC_E_INVAL, "PROLONG needs a level with a coarser level below it");
                if (!a || !out) fail(ISDC_E_INVAL, "PROLONG needs coarse input and output");
                if (per)
                    HIPCHK(launch_cprolong_p<T>(n, (const T*)a, (T*)out, s));
                else
                    HIPCHK(launch_prolong<T>(d, n, (const T*)a, (T*)out, s));
                break;
            case ISDC_OP_COARSE:
                if (n > (per ? kCTailMaxPeriodic : tail_max_n(d)))
                    fail(ISDC_E_INVAL, "COARSE level too large for one workgroup");
                if (!a || !out) fail(ISDC_E_INVAL, "COARSE needs rhs and output");
                HIPCHK(launch_ctail<T>(p->mg, n, c, p->w, h, true, (const T*)a, (T*)out, per, s));
                break;
            case ISDC_OP_RESIDUAL_NORM: {
                if (!a || !b || !h_scalar) fail(ISDC_E_INVAL, "RESIDUAL_NORM needs rhs, iterate and h_scalar");
                int nb = 0;
                HIPCHK(launch_cresnorm<T>(n, k, (const T*)a, (const T*)b, p->partial, &nb, per, s));
                HIPCHK(launch_reduce_max(p->partial, nb, p->scalars + 2, s));
                *h_scalar = read_scalar(p, p->scalars + 2, s);
                break;
            }
            default:
                fail(ISDC_E_INVAL, "unknown op");
        }
        return;
    }
    switch (op) {
        case ISDC_OP_SMOOTH: {
            if (!a || !b || !out) fail(ISDC_E_INVAL, "SMOOTH needs rhs, iterate and output");
            if (p->mg.smoother == ISDC_SMOOTH_RBGS) {
                if (out != b)  // one-pass tiled red-black step
                    HIPCHK(launch_rbgs_tile<T>(d, n, co, false, (const T*)a, (const T*)b, (T*)out, s));
                else           // in place: red and black half steps
                    HIPCHK(launch_smooth<T>(p->mg, n, co, false, (const T*)a, (const T*)out, (T*)out, s));
            } else {
                if (out == b) fail(ISDC_E_INVAL, "Jacobi SMOOTH needs a separate output array");
                HIPCHK(launch_smooth<T>(p->mg, n, co, false, (const T*)a, (const T*)b, (T*)out, s));
            }
            break;
        }
        case ISDC_OP_RESTRICT:
            if (n < 3) fail(ISDC_E_INVAL, "RESTRICT needs a level with n >= 3");
            if (!a || !b || !out) fail(ISDC_E_INVAL, "RESTRICT needs rhs, iterate and output");
            HIPCHK(launch_restrict_tile<T>(d, n, co, (const T*)a, (const T*)b, (T*)out, s));
            break;
        case ISDC_OP_PROLONG:
            if (n < 3) fail(ISDC_E_INVAL, "PROLONG needs a level with n >= 3");
            if (!a || !out) fail(ISDC_E_INVAL, "PROLONG needs coarse input and output");
            HIPCHK(launch_prolong<T>(d, n, (const T*)a, (T*)out, s));
            break;
        case ISDC_OP_COARSE:
            if (n > tail_max_n(d)) fail(ISDC_E_INVAL, "COARSE level too large for one workgroup");
            if (!a || !out) fail(ISDC_E_INVAL, "COARSE needs rhs and output");
            HIPCHK(launch_tail<T>(p->mg, n, c, h, true, (const T*)a, (T*)out, s));
            break;
        case ISDC_OP_RESIDUAL_NORM: {
            if (!a || !b || !h_scalar) fail(ISDC_E_INVAL, "RESIDUAL_NORM needs rhs, iterate and h_scalar");
            int nb = 0;
            HIPCHK(launch_resnorm<T>(d, n, co, (const T*)a, (const T*)b, p->partial, &nb, s));
            HIPCHK(launch_reduce_max(p->partial, nb, p->scalars + 2, s));
            *h_scalar = read_scalar(p, p->scalars + 2, s);
            break;
        }
        default:
            fail(ISDC_E_INVAL, "unknown op");
    }
}

}  // namespace

extern "C" int isdc_mg_op(isdc_plan* plan, int32_t op, int32_t level, double c, int32_t precision, const void* d_a,
                          const void* d_b, void* d_out, void* stream, double* h_scalar) {
    return guarded([&] {
        check_plan(plan);
        if (!std::isfinite(c) || c < 0) fail(ISDC_E_INVAL, "c must be finite and >= 0");
        if (level < 0 || level >= level_count(plan->periodic, plan->n)) fail(ISDC_E_INVAL, "level out of range");
        if (precision == ISDC_PREC_FP64)
            mg_op_impl<double>(plan, op, level, c, d_a, d_b, d_out, (hipStream_t)stream, h_scalar);
        else if (precision == ISDC_PREC_MIXED)
            mg_op_impl<float>(plan, op, level, c, d_a, d_b, d_out, (hipStream_t)stream, h_scalar);
        else
            fail(ISDC_E_INVAL, "unknown precision");
    });
}

namespace {

template <typename T>
void time_kernel_impl(isdc_plan* p, int kernel, int level, double c, int reps, hipStream_t s, double* avg_us,
                      double* bytes) {
    const int d = p->d;
    const size_t w = sizeof(T);
    std::function<void()> launch;
    double b = 0.0;
    if (p->compact) {
        // compact plans: the fused Jacobi + restriction launch (SMOOTH), the
        // compact tail and the Burgers advection
        if (kernel == ISDC_KERNEL_SMOOTH) {
            if (level < 0 || level >= p->tail) fail(ISDC_E_INVAL, "level must lie above the coarse tail for this kernel");
            const Level& L = p->lev[level];
            const CCoef<T> k = make_ccoef<T>(c, p->w, L.h, p->mg.omega);
            const bool per = p->periodic;
            // the V-cycle's fused pre-smoothing + residual + restriction launch
            const Level& Cl = p->lev[level + 1];
            const int ks = std::min(3, std::max(1, p->mg.nu_pre));
            launch = [=]() {
                HIPCHK(launch_cjres<T>(L.n, k, ks, false, (const T*)L.r, (const T*)L.e, (T*)L.e2, (T*)Cl.r, per, s));
            };
            b = (3.0 * (double)L.N + (double)Cl.N) * w;
        } else if (kernel == ISDC_KERNEL_TAIL) {
            const Level& L = p->lev[p->tail];
            launch = [=]() {
                HIPCHK(launch_ctail<T>(p->mg, L.n, c, p->w, L.h, true, (const T*)L.r, (T*)L.e, p->periodic, s));
            };
            b = 2.0 * (double)L.N * w;
        } else if (kernel == ISDC_KERNEL_EXPLICIT) {
            if (!p->fe_arrays) fail(ISDC_E_UNSUPPORTED, "ISDC_KERNEL_EXPLICIT times the WENO5 Burgers advection only");
            const Level& L = p->lev[0];
            launch = [=]() { HIPCHK(launch_weno_burgers(p->n, p->h, (const double*)L.r, (double*)L.e, s)); };
            b = 2.0 * (double)p->N * 8.0;
        } else {
            fail(ISDC_E_UNSUPPORTED, "compact plans time ISDC_KERNEL_SMOOTH, ISDC_KERNEL_TAIL and ISDC_KERNEL_EXPLICIT only");
        }
    } else {
    if (kernel != ISDC_KERNEL_TAIL && kernel != ISDC_KERNEL_QUAD && (level < 0 || level >= p->tail))
        fail(ISDC_E_INVAL, "level must lie above the coarse tail for this kernel");
    if (kernel == ISDC_KERNEL_SMOOTH_RESTRICT || kernel == ISDC_KERNEL_PROLONG_SMOOTH || kernel == ISDC_KERNEL_SMOOTH) {
        const Level& L = p->lev[level];
        const Level& C = p->lev[level + 1];
        const Coef<T> co = make_coef<T>(c, L.h, d, p->mg.omega);
        const double N = (double)L.N, Nc = (double)C.N;
        if (kernel == ISDC_KERNEL_SMOOTH_RESTRICT) {
            if (!rbgs_restrict_fused(d, L.n))
                fail(ISDC_E_UNSUPPORTED, "3D fused smoothing + restriction runs on levels of 127^3 and up");
            launch = [=]() { HIPCHK(launch_rbgs_restrict_tile<T>(d, L.n, co, false, (const T*)L.r, (const T*)L.e, (T*)L.e2, (T*)C.r, s, L.shape)); };
            b = (3.0 * N + Nc) * w;
        } else if (kernel == ISDC_KERNEL_PROLONG_SMOOTH) {
            launch = [=]() { HIPCHK(launch_prolong_rbgs_tile<T>(d, L.n, co, (const T*)L.r, (const T*)L.e2, (const T*)C.e, (T*)L.e, nullptr, nullptr, 0, s, L.shape)); };
            b = (3.0 * N + Nc) * w;
        } else {
            launch = [=]() { HIPCHK(launch_rbgs_tile<T>(d, L.n, co, false, (const T*)L.r, (const T*)L.e, (T*)L.e2, s, L.shape)); };
            b = 3.0 * N * w;
        }
    } else if (kernel == ISDC_KERNEL_TAIL) {
        const Level& L = p->lev[p->tail];
        launch = [=]() { HIPCHK(launch_tail<T>(p->mg, L.n, c, L.h, true, (const T*)L.r, (T*)L.e, s)); };
        b = 2.0 * (double)L.N * w;
    } else if (kernel == ISDC_KERNEL_QUAD) {
        if (!p->begun) fail(ISDC_E_INVAL, "ISDC_KERNEL_QUAD needs a step in progress");
        // quadrature + residual of the current iterate; S*F arrays are rewritten with the same values
        launch = [=]() { quad_residual(p, p->cur, s); };
        int reads = 1;  // u_0
        for (int j = 1; j <= p->M; ++j)
            if (p->cur[j] != p->u0) ++reads;
        int writes = 0;
        for (int m = 0; m < p->M; ++m)
            if (p->SF[m]) ++writes;
        b = (double)(reads + writes) * (double)p->N * 8.0;
    } else {
        fail(ISDC_E_INVAL, "unknown kernel");
    }
    }
    // one event pair around `reps` back-to-back launches: a pair around every
    // launch would add the events' own cost to each (a few us per launch)
    hipEvent_t ev[2];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    launch();  // warm-up
    HIPCHK(hipEventRecord(ev[0], s));
    for (int k = 0; k < reps; ++k) launch();
    HIPCHK(hipEventRecord(ev[1], s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
    for (auto& e : ev) (void)hipEventDestroy(e);
    *avg_us = (double)ms / reps * 1e3;
    *bytes = b;
}

}  // namespace

namespace {

bool level_shaped(const isdc_plan* p, int l) {
    return !p->compact && p->mg.smoother == ISDC_SMOOTH_RBGS && l < p->tail;
}

// The tiled kernels one V-cycle runs on level l (pre- and post-smoothing,
// the fused restriction and prolongation), on the plan's own buffers.
template <typename T>
void level_tile_kernels(isdc_plan* p, int l, hipStream_t s) {
    const Level& L = p->lev[l];
    const Level& C = p->lev[l + 1];
    const MGConfig& mg = p->mg;
    const Coef<T> co = make_coef<T>(1e-3, L.h, p->d, mg.omega);
    const T* r = (const T*)L.r;
    T* a = (T*)L.e;
    T* b = (T*)L.e2;
    int plain = mg.nu_pre + (mg.nu_post > 0 ? mg.nu_post - 1 : 0);
    if (rbgs_restrict_fused(p->d, L.n) && mg.nu_pre >= 1) {
        HIPCHK(launch_rbgs_restrict_tile<T>(p->d, L.n, co, false, r, a, b, (T*)C.r, s, L.shape));
        --plain;
    }
    if (mg.nu_post >= 1)
        HIPCHK(launch_prolong_rbgs_tile<T>(p->d, L.n, co, r, b, (const T*)C.e, a, nullptr, nullptr, 0, s, L.shape));
    for (int k = 0; k < plain; ++k) HIPCHK(launch_rbgs_tile<T>(p->d, L.n, co, false, r, a, b, s, L.shape));
}

// Pick each level's tile shape by timing its kernels with every shape:
// three interleaved rounds of `reps` launches per shape, the fastest round
// of each shape compared.
template <typename T>
void autotune_impl(isdc_plan* p, int reps, hipStream_t s) {
    hipEvent_t ev[2];
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (int l = 0; l < p->tail; ++l) {
        if (!level_shaped(p, l)) continue;
        double best[kTileShapes];
        for (double& b : best) b = 1e30;
        for (int round = 0; round < 3; ++round)
            for (int sh = 0; sh < kTileShapes; ++sh) {
                p->lev[l].shape = sh;
                level_tile_kernels<T>(p, l, s);  // warm-up
                HIPCHK(hipEventRecord(ev[0], s));
                for (int k = 0; k < reps; ++k) level_tile_kernels<T>(p, l, s);
                HIPCHK(hipEventRecord(ev[1], s));
                HIPCHK(hipStreamSynchronize(s));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
                best[sh] = std::min(best[sh], (double)ms);
            }
        int pick = 0;
        for (int sh = 1; sh < kTileShapes; ++sh)
            if (best[sh] < best[pick]) pick = sh;
        p->lev[l].shape = pick;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
}

void get_shapes(const isdc_plan* p, int32_t* h_shapes, int32_t max_levels, int32_t* h_nlevels) {
    if (h_nlevels) *h_nlevels = p->tail;
    if (h_shapes)
        for (int l = 0; l < p->tail && l < max_levels; ++l) h_shapes[l] = p->lev[l].shape;
}

}  // namespace

extern "C" int isdc_autotune(isdc_plan* plan, int32_t reps, void* stream, int32_t* h_shapes, int32_t max_levels,
                             int32_t* h_nlevels) {
    return guarded([&] {
        check_plan(plan);
        if (plan->begun) fail(ISDC_E_INVAL, "isdc_autotune during a step (its timing reuses the plan's buffers)");
        if (reps < 1 || reps > 10000) fail(ISDC_E_INVAL, "reps must be in 1..10000");
        if (max_levels < 0) fail(ISDC_E_INVAL, "max_levels must be >= 0");
        if (plan->par.precision == ISDC_PREC_MIXED)
            autotune_impl<float>(plan, reps, (hipStream_t)stream);
        else
            autotune_impl<double>(plan, reps, (hipStream_t)stream);
        get_shapes(plan, h_shapes, max_levels, h_nlevels);
    });
}

extern "C" int isdc_set_tile_shapes(isdc_plan* plan, const int32_t* h_shapes, int32_t nlevels) {
    return guarded([&] {
        check_plan(plan);
        if (!h_shapes && nlevels > 0) fail(ISDC_E_INVAL, "h_shapes is NULL");
        if (nlevels != plan->tail) fail(ISDC_E_INVAL, "nlevels must equal the number of levels above the tail");
        for (int l = 0; l < nlevels; ++l)
            if (h_shapes[l] < 0 || h_shapes[l] >= kTileShapes) fail(ISDC_E_INVAL, "tile shape out of range");
        for (int l = 0; l < nlevels; ++l) plan->lev[l].shape = h_shapes[l];
    });
}

extern "C" int isdc_get_tile_shapes(const isdc_plan* plan, int32_t* h_shapes, int32_t max_levels,
                                    int32_t* h_nlevels) {
    return guarded([&] {
        check_plan(plan);
        if (max_levels < 0) fail(ISDC_E_INVAL, "max_levels must be >= 0");
        get_shapes(plan, h_shapes, max_levels, h_nlevels);
    });
}

extern "C" int isdc_time_kernel(isdc_plan* plan, int32_t kernel, int32_t level, double c, int32_t precision,
                                int32_t reps, void* stream, double* h_avg_us, double* h_bytes) {
    return guarded([&] {
        check_plan(plan);
        if (!std::isfinite(c) || c < 0) fail(ISDC_E_INVAL, "c must be finite and >= 0");
        if (reps < 1 || reps > 100000) fail(ISDC_E_INVAL, "reps must be in 1..100000");
        if (!h_avg_us || !h_bytes) fail(ISDC_E_INVAL, "NULL output");
        if (precision == ISDC_PREC_FP64)
            time_kernel_impl<double>(plan, kernel, level, c, reps, (hipStream_t)stream, h_avg_us, h_bytes);
        else if (precision == ISDC_PREC_MIXED)
            time_kernel_impl<float>(plan, kernel, level, c, reps, (hipStream_t)stream, h_avg_us, h_bytes);
        else
            fail(ISDC_E_INVAL, "unknown precision");
    });
}
