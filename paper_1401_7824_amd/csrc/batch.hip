// Batched ISDC: many independent instances ("slots") advanced sweep by sweep
// together, with one kernel launch per phase of the sweep for all of them.
//
// Each slot is an ordinary plan (its own workspace and multigrid hierarchy;
// grid size, nu, dt, M, node family and tolerance may differ between slots).
// A launch covers the tiles of every participating slot: workgroup b finds
// its slot and tile in a compact (slot, first tile) map by binary search and
// runs the same device body as the single-instance kernel, with the same
// coefficients, so a slot's result is bitwise the result of isdc_step.
//
// Sweep schedule (eq. (4), Sec. 3) for substep phase p = 0.. max over slots
// of the number of non-degenerate substeps: right-hand side; then for each
// of the L V-cycles the down legs of level 0, 1, ... (levels aligned from the
// finest), one coarse-tail workgroup per slot, and the up legs back to level
// 0 (the last one writing the node value); finally the quadrature + SDC
// residual of every slot and one residual per slot to the host.  Slots join
// (begin a step) and leave (end a step, converge, fail) between sweeps.
#include <hip/hip_runtime.h>

#include <chrono>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "jrows.h"
#include "mg_device.h"
#include "mg_march.h"
#include "plan.h"
#include "rows2d.h"
#include "tailc.h"
#include "sdc_device.h"

namespace isdc {
namespace {

constexpr int kMaxLev = 16;
using BRow = RowShape<0>::RT;  // the row tile of 2D levels
constexpr int kChunkPts = 4 * kThreads;  // points per workgroup of the pointwise kernels

struct SlotDesc {
    int n, nlev, ns, M, fe, N;
    int sub[ISDC_MAX_M];     // substep m of substep phase p
    double dtm[ISDC_MAX_M];  // dt_m of phase p
    int ln[kMaxLev];         // interior points per axis of each level (nlev = the tail level)
    void* lr[kMaxLev];
    void* le[kMaxLev];
    void* le2[kMaxLev];
    double la[ISDC_MAX_M][kMaxLev], ldiag[ISDC_MAX_M][kMaxLev], linv[ISDC_MAX_M][kMaxLev];
    TailCoefs tail[ISDC_MAX_M];
    // weighted-Jacobi V(jpre, jpost) cycles (jac = 1; 2D): the five-point
    // operator's coefficients (make_coef5) per phase and level, and omega
    int jac, jpre, jpost;
    double jomega;
    double jb0[ISDC_MAX_M][kMaxLev], jbf[ISDC_MAX_M][kMaxLev], jinv[ISDC_MAX_M][kMaxLev];
    double* ustate;                // u_0 of the current step; receives u_M at its end
    double* U[2][ISDC_MAX_M + 1];  // node j of buffer b (j = 0, and j = 1 for Gauss-Lobatto: ustate)
    double* SF[ISDC_MAX_M];
    QuadArgs qa[3];                // quadrature over buffer 0, buffer 1, or over u_0 at every node
    double* partial;
    int quad_tiles;
};

struct SlotState {
    int parity;  // buffer written by the current / most recent sweep
    int pad;
};

struct BArgs {
    const SlotDesc* desc;
    const SlotState* st;
    const int* map;  // [count, slot[count], first tile[count]]
    int p, level, flag;
    double* out;
};

__device__ __forceinline__ void map_lookup(const int* map, int& slot, int& t) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int cnt = map[0];
    const int* sl = map + 1;
    const int* first = map + 1 + cnt;
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    slot = sl[lo];
    t = b - first[lo];
}

template <int D>
__device__ __forceinline__ void tile_xyz(int t, int n, int TX, int TY, int TZ, int& x0, int& y0, int& z0) {
    const int ntx = (n + TX - 1) / TX;
    const int nty = D >= 2 ? (n + TY - 1) / TY : 1;
    const int tx = t % ntx;
    const int r = t / ntx;
    x0 = tx * TX;
    y0 = (r % nty) * TY;
    z0 = (r / nty) * TZ;
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) kb_rhs(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int par = a.st[i].parity;
    const int m = s.sub[a.p];
    const double* umn = s.U[par][m];
    const double* umo = s.U[par ^ 1][m];
    const double* upo = s.U[par ^ 1][m + 1];
    const double* sf = s.SF[m];
    T* r = (T*)s.lr[0];
    const double dtm = s.dtm[a.p];
#pragma unroll
    for (int q = 0; q < kChunkPts / kThreads; ++q) {
        const int k = t * kChunkPts + q * kThreads + threadIdx.x;
        if (k < s.N) {
            const double base = umn[k] + dtm * (fexp(umn[k], s.fe) - fexp(umo[k], s.fe)) + sf[k];
            r[k] = T(base - upo[k]);
        }
    }
}

template <typename T, int D, bool ZERO>
__global__ void __launch_bounds__(kThreads) kb_rbgs_restrict(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int x0, y0, z0;
    if constexpr (D == 2) {
        tile_xyz<D>(t, s.ln[l], BRow::TX, BRow::TY, 1, x0, y0, z0);
        rows_rbgs_restrict_body<T, ZERO, BRow>((const T*)s.lr[l], (const T*)s.le[l], (T*)s.le2[l], (T*)s.lr[l + 1],
                                               s.ln[l], x0, y0, T(s.la[p][l]), T(s.ldiag[p][l]), T(s.linv[p][l]));
    } else {
        tile_xyz<D>(t, s.ln[l], Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
        rbgs_restrict_body<T, D, ZERO>((const T*)s.lr[l], (const T*)s.le[l], (T*)s.le2[l], (T*)s.lr[l + 1], s.ln[l],
                                       x0, y0, z0, T(s.la[p][l]), T(s.ldiag[p][l]), T(s.linv[p][l]));
    }
}

template <typename T, int D, bool ZERO>
__global__ void __launch_bounds__(kThreads) kb_rbgs(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int x0, y0, z0;
    const int mz = D == 3 ? march_depth(s.ln[l]) : 0;
    if constexpr (D == 2) {
        tile_xyz<D>(t, s.ln[l], BRow::TX, BRow::TY, 1, x0, y0, z0);
        rows_rbgs_body<T, ZERO, BRow>((const T*)s.lr[l], (const T*)s.le[l], (T*)s.le2[l], s.ln[l], x0, y0,
                                      T(s.la[p][l]), T(s.linv[p][l]));
    } else if (D == 3 && mz > 0) {
        tile_xyz<D>(t, s.ln[l], MTile<T>::X, MTile<T>::Y, mz, x0, y0, z0);
        march_rbgs_body<T, false, 0, ZERO>((const T*)s.lr[l], (const T*)s.le[l], nullptr, (T*)s.le2[l], s.ln[l], x0, y0,
                                           z0, mz, T(s.la[p][l]), T(s.linv[p][l]), nullptr, nullptr);
    } else {
        tile_xyz<D>(t, s.ln[l], Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
        rbgs_tile_body<T, D, ZERO>((const T*)s.lr[l], (const T*)s.le[l], (T*)s.le2[l], s.ln[l], x0, y0, z0,
                                   T(s.la[p][l]), T(s.linv[p][l]));
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads) kb_restrict(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int X0, Y0, Z0;
    if (D == 3 && march_depth(s.ln[l]) > 0) {
        tile_xyz<D>(t, (s.ln[l] - 1) / 2, MRTile::X, MRTile::Y, march_restrict_depth(), X0, Y0, Z0);
        march_restrict_body<T>((const T*)s.lr[l], (const T*)s.le2[l], (T*)s.lr[l + 1], s.ln[l], X0, Y0, Z0,
                               march_restrict_depth(), T(s.la[p][l]), T(s.ldiag[p][l]));
        return;
    }
    tile_xyz<D>(t, (s.ln[l] - 1) / 2, CTile<D>::X, CTile<D>::Y, CTile<D>::Z, X0, Y0, Z0);
    restrict_tile_body<T, D>((const T*)s.lr[l], (const T*)s.le2[l], (T*)s.lr[l + 1], s.ln[l], X0, Y0, Z0,
                             T(s.la[p][l]), T(s.ldiag[p][l]));
}

template <typename T, int D>
__global__ void __launch_bounds__(kTail) kb_tail(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = s.nlev;
    // the tail starts from zero below the finest level and in the first cycle
    const int zero = (a.flag == 0 || l > 0) ? 1 : 0;
    if (s.jac)
        tailc_body<T, D>((const T*)s.lr[l], (T*)s.le[l], s.ln[l], s.tail[a.p], ISDC_SMOOTH_JACOBI, s.jpre, s.jpost,
                         s.jomega, zero);
    else
        tailc_body<T, D>((const T*)s.lr[l], (T*)s.le[l], s.ln[l], s.tail[a.p], ISDC_SMOOTH_RBGS, 1, 1, 0.0, zero);
}

// 2D weighted-Jacobi cycles, as the single-instance fused row kernels: K
// steps + residual + full weighting (e: le -> le2, coarse rhs: lr[l+1]) ...
template <typename T, int K, bool ZERO>
__global__ void __launch_bounds__(kThreads) kb_jres(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int x0, y0, z0;
    tile_xyz<2>(t, s.ln[l], CVT<K>::TX, CVT<K>::TY, 1, x0, y0, z0);
    const CCoef<T> k{T(s.jb0[p][l]), T(s.jbf[p][l]), T(0), T(s.jinv[p][l]), T(s.jomega)};
    cjres_tile<T, false, K, ZERO, false>((const T*)s.lr[l], (const T*)s.le[l], (T*)s.le2[l], (T*)s.lr[l + 1], s.ln[l],
                                        x0, y0, k);
}

// ... and prolongation + correction + K steps (le2 + P le[l+1] -> le; MODE 1:
// the node value g + e to the sweep's node array instead)
template <typename T, int K, int MODE>
__global__ void __launch_bounds__(kThreads) kb_pjac(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int x0, y0, z0;
    tile_xyz<2>(t, s.ln[l], CVT<K>::TX, CVT<K>::TY, 1, x0, y0, z0);
    const int par = a.st[i].parity, m = s.sub[p];
    const double* g = MODE == 1 ? s.U[par ^ 1][m + 1] : nullptr;
    double* u_out = MODE == 1 ? s.U[par][m + 1] : nullptr;
    const CCoef<T> k{T(s.jb0[p][l]), T(s.jbf[p][l]), T(0), T(s.jinv[p][l]), T(s.jomega)};
    cpjac_tile<T, false, K, false, MODE>((const T*)s.lr[l], (const T*)s.le2[l], (const T*)s.le[l + 1], (T*)s.le[l],
                                         s.ln[l], x0, y0, k, g, u_out);
}

template <typename T, int D, int MODE>
__global__ void __launch_bounds__(kThreads) kb_prolong_rbgs(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int l = a.level, p = a.p;
    int x0, y0, z0;
    const int par = a.st[i].parity, m = s.sub[p];
    const double* g = MODE == 1 ? s.U[par ^ 1][m + 1] : nullptr;
    double* u_out = MODE == 1 ? s.U[par][m + 1] : nullptr;
    const int mz = D == 3 ? march_depth(s.ln[l]) : 0;
    if constexpr (D == 2) {
        tile_xyz<D>(t, s.ln[l], BRow::TX, BRow::TY, 1, x0, y0, z0);
        rows_prolong_rbgs_body<T, MODE, BRow>((const T*)s.lr[l], (const T*)s.le2[l], (const T*)s.le[l + 1],
                                              (T*)s.le[l], s.ln[l], x0, y0, T(s.la[p][l]), T(s.linv[p][l]), g, u_out);
    } else if (D == 3 && mz > 0) {
        tile_xyz<D>(t, s.ln[l], MTile<T>::X, MTile<T>::Y, mz, x0, y0, z0);
        march_rbgs_body<T, true, MODE, false>((const T*)s.lr[l], (const T*)s.le2[l], (const T*)s.le[l + 1],
                                              (T*)s.le[l], s.ln[l], x0, y0, z0, mz, T(s.la[p][l]), T(s.linv[p][l]), g,
                                              u_out);
    } else {
        tile_xyz<D>(t, s.ln[l], Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
        prolong_rbgs_body<T, D, MODE>((const T*)s.lr[l], (const T*)s.le2[l], (const T*)s.le[l + 1], (T*)s.le[l],
                                      s.ln[l], x0, y0, z0, T(s.la[p][l]), T(s.linv[p][l]), g, u_out);
    }
}

// u_{m+1}^{k+1} = u_{m+1}^k + e for slots whose finest level is the tail.
template <typename T>
__global__ void __launch_bounds__(kThreads) kb_update(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    const int par = a.st[i].parity, m = s.sub[a.p];
    const double* g = s.U[par ^ 1][m + 1];
    double* out = s.U[par][m + 1];
    const T* e = (const T*)s.le[0];
#pragma unroll
    for (int q = 0; q < kChunkPts / kThreads; ++q) {
        const int k = t * kChunkPts + q * kThreads + threadIdx.x;
        if (k < s.N) out[k] = g[k] + (double)e[k];
    }
}

template <int D, int M>
__global__ void __launch_bounds__(kThreads) kb_quad(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    int x0, y0, z0;
    tile_xyz<D>(t, s.n, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
    const QuadArgs& qa = s.qa[a.flag ? 2 : a.st[i].parity];
    const double mx = quad_residual_body<D, M>(qa, x0, y0, z0);
    if (threadIdx.x == 0) s.partial[t] = mx;
}

__global__ void __launch_bounds__(kThreads) kb_reduce(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
    double m = 0.0;
    for (int k = threadIdx.x; k < s.quad_tiles; k += kThreads) m = nanmax(m, s.partial[k]);
    m = block_max(m);
    if (threadIdx.x == 0) a.out[i] = m;
}

// flag 0: spread u_0 to the nodes of buffer 0; flag 1: u_state = u_M of the
// buffer written last.
__global__ void __launch_bounds__(kThreads) kb_copy(BArgs a) {
    int i, t;
    map_lookup(a.map, i, t);
    const SlotDesc& s = a.desc[i];
#pragma unroll
    for (int q = 0; q < kChunkPts / kThreads; ++q) {
        const int k = t * kChunkPts + q * kThreads + threadIdx.x;
        if (k >= s.N) continue;
        if (a.flag == 0) {
            const double v = s.ustate[k];
            for (int j = 1; j <= s.M; ++j)
                if (s.U[0][j] != s.ustate) s.U[0][j][k] = v;
        } else {
            s.ustate[k] = s.U[a.st[i].parity][s.M][k];
        }
    }
}

// ---------------------------------------------------------------- host side

enum { SLOT_FREE = 0, SLOT_RUNNING = 1, SLOT_FINISHED = 2 };

struct Slot {
    int state = SLOT_FREE;
    isdc_plan* plan = nullptr;
    double* u = nullptr;
    double dt = 0.0;
    int nsteps = 0, steps_done = 0;
    bool need_begin = false;
    bool need_end = false;
    int parity = 0;
    int status = ISDC_OK;
    isdc_stats cur{}, last{};
    int64_t vcycles_total = 0;
};

struct Map {
    std::vector<int> slots, first;
    int total = 0;
    void add(int slot, int ntiles) {
        if (ntiles <= 0) return;
        slots.push_back(slot);
        first.push_back(total);
        total += ntiles;
    }
};

}  // namespace
}  // namespace isdc

struct isdc_batch {
    int cap, d, prec, L;
    // device (caller's workspace)
    isdc::SlotDesc* d_desc;
    isdc::SlotState* d_state;
    double* d_res;
    int* d_maps;
    size_t maps_cap;  // ints
    // pinned host staging
    isdc::SlotDesc* h_desc;
    isdc::SlotState* h_state[2];
    double* h_res;
    int* h_maps;
    std::vector<bool> desc_dirty;
    std::vector<isdc::Slot> slots;
    // instances fixed at creation (isdc_batch_create): problem, parameters and
    // plan workspace per slot, carved from the caller's one workspace
    bool fixed = false;
    std::vector<isdc_problem> fprob;
    std::vector<isdc_params> fpar;
    std::vector<char*> fws;
    std::vector<size_t> fbytes;
};

namespace isdc {
namespace {

size_t batch_layout(int cap, char* base, isdc_batch* b) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        void* p = base ? (void*)(base + off) : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    void* desc = take((size_t)cap * sizeof(SlotDesc));
    void* st = take((size_t)cap * sizeof(SlotState));
    void* res = take((size_t)cap * sizeof(double));
    const size_t maps_cap = (size_t)400 * (2 * (size_t)cap + 2);
    void* maps = take(maps_cap * sizeof(int));
    if (b) {
        b->d_desc = (SlotDesc*)desc;
        b->d_state = (SlotState*)st;
        b->d_res = (double*)res;
        b->d_maps = (int*)maps;
        b->maps_cap = maps_cap;
    }
    return off;
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }


template <int D>
int ntiles_of(int n, int TX, int TY, int TZ) {
    int c = ceil_div(n, TX);
    if (D >= 2) c *= ceil_div(n, TY);
    if (D == 3) c *= ceil_div(n, TZ);
    return c;
}

int tiles_fine(int d, int n) {
    return d == 1 ? ntiles_of<1>(n, Tile<1>::X, 1, 1)
                  : (d == 2 ? ntiles_of<2>(n, Tile<2>::X, Tile<2>::Y, 1)
                            : ntiles_of<3>(n, Tile<3>::X, Tile<3>::Y, Tile<3>::Z));
}

// Workgroups of the smoothing kernels on an n^d level (3D: marched columns,
// 2D: row-mapped tiles).
int tiles_smooth(int d, int n, bool fp64) {
    if (d == 2) return ntiles_of<2>(n, BRow::TX, BRow::TY, 1);
    if (d == 3 && march_depth(n) > 0)
        return fp64 ? ntiles_of<3>(n, MTile<double>::X, MTile<double>::Y, march_depth(n))
                    : ntiles_of<3>(n, MTile<float>::X, MTile<float>::Y, march_depth(n));
    return tiles_fine(d, n);
}

// Workgroups of the 2D weighted-Jacobi kernels with K steps on an n^2 level.
int tiles_jac(int K, int n) {
    switch (K) {
        case 1: return ntiles_of<2>(n, CVT<1>::TX, CVT<1>::TY, 1);
        case 2: return ntiles_of<2>(n, CVT<2>::TX, CVT<2>::TY, 1);
        default: return ntiles_of<2>(n, CVT<3>::TX, CVT<3>::TY, 1);
    }
}

int tiles_coarse(int d, int nc) {
    if (d == 3 && march_depth(2 * nc + 1) > 0)  // the fine level is marched: so is its restriction
        return ntiles_of<3>(nc, MRTile::X, MRTile::Y, march_restrict_depth());
    return d == 1 ? ntiles_of<1>(nc, CTile<1>::X, 1, 1)
                  : (d == 2 ? ntiles_of<2>(nc, CTile<2>::X, CTile<2>::Y, 1)
                            : ntiles_of<3>(nc, CTile<3>::X, CTile<3>::Y, CTile<3>::Z));
}

void check_batch_params(const isdc_batch* b, const isdc_problem* pb, const isdc_params* pr) {
    if (pb->dim != b->d) fail(ISDC_E_INVAL, "slot dimension differs from the batch's");
    if (pb->stencil != ISDC_STENCIL_2ND) fail(ISDC_E_UNSUPPORTED, "batches run the second-order stencil only");
    if (pb->bc != ISDC_BC_DIRICHLET) fail(ISDC_E_UNSUPPORTED, "batches run Dirichlet problems only");
    if (pr->node_kind == ISDC_NODES_LEGENDRE)
        fail(ISDC_E_UNSUPPORTED, "batches run node families that end on tau_M = 1 only");
    if (pr->precision != b->prec) fail(ISDC_E_INVAL, "slot precision differs from the batch's");
    if (pr->vcycles != b->L) fail(ISDC_E_INVAL, "slot vcycles differs from the batch's");
    const bool rb11 = pr->smoother == ISDC_SMOOTH_RBGS && pr->nu_pre == 1 && pr->nu_post == 1;
    const bool jac = b->d == 2 && pr->smoother == ISDC_SMOOTH_JACOBI && pr->nu_pre >= 1 && pr->nu_pre <= 3 &&
                     pr->nu_post >= 1 && pr->nu_post <= 3;
    if (!rb11 && !jac)
        fail(ISDC_E_UNSUPPORTED,
             "batches run red-black Gauss-Seidel V(1,1) cycles, or in 2D weighted-Jacobi V(nu1, nu2) cycles with "
             "1 <= nu1, nu2 <= 3");
    if (pr->guess != ISDC_GUESS_PREV_SWEEP) fail(ISDC_E_UNSUPPORTED, "batches warm-start from the previous sweep only");
    if (pr->early_exit) fail(ISDC_E_UNSUPPORTED, "batches run exactly L cycles per solve");
    if (pr->levels != 1) fail(ISDC_E_UNSUPPORTED, "batches run single-level ISDC only");
}

// isdc_batch_create's workspace: the batch arrays, then each instance's plan
// workspace (validated and checked against the batch rules).
size_t fixed_layout(int count, const isdc_problem* probs, const isdc_params* pars, char* base, isdc_batch* b) {
    size_t off = batch_layout(count, nullptr, nullptr);
    if (b) {
        b->fws.assign(count, nullptr);
        b->fbytes.assign(count, 0);
    }
    isdc_batch shape{};
    shape.d = probs[0].dim;
    shape.prec = pars[0].precision;
    shape.L = pars[0].vcycles;
    for (int i = 0; i < count; ++i) {
        validate(&probs[i], &pars[i]);
        if (shape.L < 1) fail(ISDC_E_UNSUPPORTED, "batches run a fixed number L >= 1 of V-cycles per solve");
        check_batch_params(&shape, &probs[i], &pars[i]);
        const size_t need = layout(probs[i], pars[i], nullptr, nullptr);
        if (b) {
            b->fws[i] = base + off;
            b->fbytes[i] = need;
        }
        off = align_up(off + need);
    }
    return off;
}

void build_desc(isdc_batch* b, int slot) {
    Slot& sl = b->slots[slot];
    const isdc_plan* p = sl.plan;
    SlotDesc& s = b->h_desc[slot];
    std::memset(&s, 0, sizeof(s));
    s.n = p->n;
    s.nlev = p->tail;
    s.M = p->M;
    s.fe = p->prob.fe_kind;
    s.N = (int)p->N;
    int ns = 0;
    for (int m = 0; m < p->M; ++m)
        if (p->dtau[m] != 0.0) {
            s.sub[ns] = m;
            s.dtm[ns] = sl.dt * p->dtau[m];
            ++ns;
        }
    s.ns = ns;
    for (size_t l = 0; l < p->lev.size(); ++l) {
        s.ln[l] = p->lev[l].n;
        s.lr[l] = p->lev[l].r;
        s.le[l] = p->lev[l].e;
        s.le2[l] = p->lev[l].e2;
    }
    for (int q = 0; q < ns; ++q) {
        const double c = s.dtm[q] * p->prob.nu;
        for (int l = 0; l < p->tail; ++l) {
            const Coef<double> co = make_coef<double>(c, p->lev[l].h, p->d, p->mg.omega);
            s.la[q][l] = co.a;
            s.ldiag[q][l] = co.diag;
            s.linv[q][l] = co.invdiag;
        }
        if (p->mg.smoother == ISDC_SMOOTH_JACOBI)
            for (int l = 0; l < p->tail; ++l) {  // as the single-instance 2D Jacobi cycle forms them
                const CCoef<double> k5 = make_coef5<double>(c, p->lev[l].h, p->mg.omega);
                s.jb0[q][l] = k5.b0;
                s.jbf[q][l] = k5.bf;
                s.jinv[q][l] = k5.inv_b0;
            }
        // the tail's level coefficients, exactly as the single-instance launcher forms them
        double hl = p->lev[p->tail].h;
        for (int l = 0, m = p->lev[p->tail].n; l < 16; ++l, m = (m - 1) / 2, hl *= 2.0) {
            const Coef<double> co = make_coef<double>(c, hl, p->d, p->mg.omega);
            s.tail[q].a[l] = co.a;
            s.tail[q].diag[l] = co.diag;
            s.tail[q].invdiag[l] = co.invdiag;
            if (m == 1) break;
        }
    }
    s.jac = p->mg.smoother == ISDC_SMOOTH_JACOBI ? 1 : 0;
    s.jpre = p->mg.nu_pre;
    s.jpost = p->mg.nu_post;
    s.jomega = p->mg.omega;
    s.ustate = sl.u;
    for (int bf = 0; bf < 2; ++bf) {
        s.U[bf][0] = sl.u;
        for (int j = 1; j <= p->M; ++j) s.U[bf][j] = p->U[bf][j] ? p->U[bf][j] : sl.u;
    }
    for (int m = 0; m < p->M; ++m) s.SF[m] = p->SF[m];
    for (int v = 0; v < 3; ++v) {
        QuadArgs& qa = s.qa[v];
        qa.u[0] = sl.u;
        for (int j = 1; j <= p->M; ++j) qa.u[j] = v == 2 ? sl.u : s.U[v][j];
        for (int m = 0; m < p->M; ++m) {
            qa.sf[m] = p->SF[m];
            for (int j = 0; j < p->M; ++j) {
                qa.dtS[m * ISDC_MAX_M + j] = sl.dt * p->S[m * p->M + j];
                qa.dtQ[m * ISDC_MAX_M + j] = sl.dt * p->Q[m * p->M + j];
            }
        }
        qa.nu_h2 = p->prob.nu / (p->h * p->h);
        qa.M = p->M;
        qa.n = p->n;
        qa.fe = p->prob.fe_kind;
    }
    s.partial = p->partial;
    s.quad_tiles = tiles_fine(p->d, p->n);
    b->desc_dirty[slot] = true;
}

// Host staging of maps: appended to h_maps, uploaded once, addressed by offset.
struct MapBuf {
    isdc_batch* b;
    size_t used = 0;
    size_t put(const Map& m) {
        const size_t need = 1 + 2 * m.slots.size();
        if (used + need > b->maps_cap) fail(ISDC_E_WORKSPACE, "batch map buffer exhausted");
        const size_t off = used;
        int* h = b->h_maps + off;
        h[0] = (int)m.slots.size();
        for (size_t k = 0; k < m.slots.size(); ++k) {
            h[1 + k] = m.slots[k];
            h[1 + m.slots.size() + k] = m.first[k];
        }
        used += need;
        return off;
    }
};

#define ISDC_BLAUNCH(kernel, threads, m, off, ...)                                                   \
    do {                                                                                             \
        if ((m).total > 0) {                                                                         \
            hipLaunchKernelGGL(kernel, dim3((m).total), dim3(threads), 0, s, __VA_ARGS__);           \
            HIPCHK(hipGetLastError());                                                               \
        }                                                                                            \
    } while (0)

template <int D>
void launch_quad_m(int M, const Map& m, BArgs a, hipStream_t s) {
    switch (M) {
#define ISDC_QBM(MM) \
    case MM: ISDC_BLAUNCH((kb_quad<D, MM>), kThreads, m, 0, a); break;
        ISDC_QBM(1) ISDC_QBM(2) ISDC_QBM(3) ISDC_QBM(4) ISDC_QBM(5) ISDC_QBM(6) ISDC_QBM(7) ISDC_QBM(8) ISDC_QBM(9)
#undef ISDC_QBM
        default: fail(ISDC_E_INVAL, "M out of range");
    }
}

// Sweep timing request of isdc_batch_time_sweeps.
struct SweepTiming {
    int reps;
    bool graph;
    double us;
    int launches;
};

// One batch sweep for the running slots (plus the begins and ends around it).
template <typename T, int D>
void advance_impl(isdc_batch* b, hipStream_t s, std::vector<int>& run, SweepTiming* timing = nullptr) {
    const int cap = b->cap;
    // upload descriptors that changed
    for (int i = 0; i < cap; ++i)
        if (b->desc_dirty[i]) {
            HIPCHK(hipMemcpyAsync(b->d_desc + i, b->h_desc + i, sizeof(SlotDesc), hipMemcpyHostToDevice, s));
            b->desc_dirty[i] = false;
        }
    MapBuf mb{b};
    // ---- begins: spread u_0 and form S F(u_0)
    Map mbeg;
    std::vector<Map> mqb(ISDC_MAX_M + 1);
    for (int i : run)
        if (b->slots[i].need_begin) {
            const isdc_plan* p = b->slots[i].plan;
            mbeg.add(i, ceil_div((int)p->N, kChunkPts));
            mqb[p->M].add(i, tiles_fine(D, p->n));
        }
    // ---- sweep maps
    int maxns = 0, maxlev = 0;
    for (int i : run) {
        maxns = std::max(maxns, b->h_desc[i].ns);
        maxlev = std::max(maxlev, b->h_desc[i].nlev);
    }
    std::vector<Map> mrhs(maxns), mtail(maxns), mupd(maxns);
    std::vector<std::vector<Map>> mlev(maxns, std::vector<Map>(maxlev)), mres(maxns, std::vector<Map>(maxlev));
    // 2D weighted-Jacobi slots by number of steps K (1..3): pre- and post-smoothing launches
    std::vector<std::vector<std::vector<Map>>> mjres(4, std::vector<std::vector<Map>>(maxns, std::vector<Map>(maxlev)));
    std::vector<std::vector<std::vector<Map>>> mpjac(4, std::vector<std::vector<Map>>(maxns, std::vector<Map>(maxlev)));
    std::vector<Map> mq(ISDC_MAX_M + 1);
    Map mred;
    for (int i : run) {
        const SlotDesc& sd = b->h_desc[i];
        for (int p = 0; p < sd.ns; ++p) {
            mrhs[p].add(i, ceil_div(sd.N, kChunkPts));
            mtail[p].add(i, 1);
            if (sd.nlev == 0) mupd[p].add(i, ceil_div(sd.N, kChunkPts));
            for (int l = 0; l < sd.nlev; ++l) {
                if (D == 2 && sd.jac) {
                    mjres[sd.jpre][p][l].add(i, tiles_jac(sd.jpre, sd.ln[l]));
                    mpjac[sd.jpost][p][l].add(i, tiles_jac(sd.jpost, sd.ln[l]));
                    continue;
                }
                mlev[p][l].add(i, tiles_smooth(D, sd.ln[l], b->prec == ISDC_PREC_FP64));
                mres[p][l].add(i, tiles_coarse(D, (sd.ln[l] - 1) / 2));
            }
        }
        mq[sd.M].add(i, sd.quad_tiles);
        mred.add(i, 1);
    }
    const size_t o_beg = mb.put(mbeg);
    std::vector<size_t> o_qb(ISDC_MAX_M + 1), o_q(ISDC_MAX_M + 1);
    for (int M = 1; M <= ISDC_MAX_M; ++M) {
        o_qb[M] = mb.put(mqb[M]);
        o_q[M] = mb.put(mq[M]);
    }
    std::vector<size_t> o_rhs(maxns), o_tail(maxns), o_upd(maxns);
    std::vector<std::vector<size_t>> o_lev(maxns, std::vector<size_t>(maxlev)), o_res(maxns, std::vector<size_t>(maxlev));
    std::vector<std::vector<std::vector<size_t>>> o_jres(4, std::vector<std::vector<size_t>>(maxns, std::vector<size_t>(maxlev)));
    std::vector<std::vector<std::vector<size_t>>> o_pjac(4, std::vector<std::vector<size_t>>(maxns, std::vector<size_t>(maxlev)));
    for (int p = 0; p < maxns; ++p) {
        o_rhs[p] = mb.put(mrhs[p]);
        o_tail[p] = mb.put(mtail[p]);
        o_upd[p] = mb.put(mupd[p]);
        for (int l = 0; l < maxlev; ++l) {
            o_lev[p][l] = mb.put(mlev[p][l]);
            o_res[p][l] = mb.put(mres[p][l]);
            for (int K = 1; K <= 3; ++K) {
                if (mjres[K][p][l].total) o_jres[K][p][l] = mb.put(mjres[K][p][l]);
                if (mpjac[K][p][l].total) o_pjac[K][p][l] = mb.put(mpjac[K][p][l]);
            }
        }
    }
    const size_t o_red = mb.put(mred);
    HIPCHK(hipMemcpyAsync(b->d_maps, b->h_maps, mb.used * sizeof(int), hipMemcpyHostToDevice, s));
    // states for the sweep: begun slots write buffer 1 first
    SlotState* hs = b->h_state[0];
    for (int i : run) {
        if (b->slots[i].need_begin) b->slots[i].parity = 1;
        hs[i].parity = b->slots[i].parity;
    }
    HIPCHK(hipMemcpyAsync(b->d_state, hs, cap * sizeof(SlotState), hipMemcpyHostToDevice, s));
    auto A = [&](size_t off, int p, int level, int flag) {
        return BArgs{b->d_desc, b->d_state, b->d_maps + off, p, level, flag, b->d_res};
    };
    ISDC_BLAUNCH(kb_copy, kThreads, mbeg, 0, A(o_beg, 0, 0, 0));
    for (int M = 1; M <= ISDC_MAX_M; ++M)
        if (mqb[M].total) launch_quad_m<D>(M, mqb[M], A(o_qb[M], 0, 0, 1), s);
    for (int i : run) b->slots[i].need_begin = false;
    // ---- the sweep
    const int L = b->L;
    auto sweep = [&]() {
    for (int p = 0; p < maxns; ++p) {
        ISDC_BLAUNCH((kb_rhs<T, D>), kThreads, mrhs[p], 0, A(o_rhs[p], p, 0, 0));
        for (int c = 0; c < L; ++c) {
            for (int l = 0; l < maxlev; ++l) {
                const bool zero = c == 0 || l > 0;
                if (D <= 2) {
                    if (zero) ISDC_BLAUNCH((kb_rbgs_restrict<T, D, true>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                    else ISDC_BLAUNCH((kb_rbgs_restrict<T, D, false>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                    if constexpr (D == 2)
                        for (int K = 1; K <= 3; ++K) {
                            const Map& m = mjres[K][p][l];
                            if (!m.total) continue;
                            const BArgs ba = A(o_jres[K][p][l], p, l, 0);
                            if (K == 1 && zero) ISDC_BLAUNCH((kb_jres<T, 1, true>), kThreads, m, 0, ba);
                            else if (K == 1) ISDC_BLAUNCH((kb_jres<T, 1, false>), kThreads, m, 0, ba);
                            else if (K == 2 && zero) ISDC_BLAUNCH((kb_jres<T, 2, true>), kThreads, m, 0, ba);
                            else if (K == 2) ISDC_BLAUNCH((kb_jres<T, 2, false>), kThreads, m, 0, ba);
                            else if (zero) ISDC_BLAUNCH((kb_jres<T, 3, true>), kThreads, m, 0, ba);
                            else ISDC_BLAUNCH((kb_jres<T, 3, false>), kThreads, m, 0, ba);
                        }
                } else {
                    if (zero) ISDC_BLAUNCH((kb_rbgs<T, D, true>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                    else ISDC_BLAUNCH((kb_rbgs<T, D, false>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                    ISDC_BLAUNCH((kb_restrict<T, D>), kThreads, mres[p][l], 0, A(o_res[p][l], p, l, 0));
                }
            }
            ISDC_BLAUNCH((kb_tail<T, D>), kTail, mtail[p], 0, A(o_tail[p], p, 0, c));
            for (int l = maxlev - 1; l >= 0; --l) {
                const bool upd = l == 0 && c == L - 1;  // the node update u = g + e in the last launch
                if (upd)
                    ISDC_BLAUNCH((kb_prolong_rbgs<T, D, 1>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                else
                    ISDC_BLAUNCH((kb_prolong_rbgs<T, D, 0>), kThreads, mlev[p][l], 0, A(o_lev[p][l], p, l, 0));
                if constexpr (D == 2)
                    for (int K = 1; K <= 3; ++K) {
                        const Map& m = mpjac[K][p][l];
                        if (!m.total) continue;
                        const BArgs ba = A(o_pjac[K][p][l], p, l, 0);
                        if (K == 1 && upd) ISDC_BLAUNCH((kb_pjac<T, 1, 1>), kThreads, m, 0, ba);
                        else if (K == 1) ISDC_BLAUNCH((kb_pjac<T, 1, 0>), kThreads, m, 0, ba);
                        else if (K == 2 && upd) ISDC_BLAUNCH((kb_pjac<T, 2, 1>), kThreads, m, 0, ba);
                        else if (K == 2) ISDC_BLAUNCH((kb_pjac<T, 2, 0>), kThreads, m, 0, ba);
                        else if (upd) ISDC_BLAUNCH((kb_pjac<T, 3, 1>), kThreads, m, 0, ba);
                        else ISDC_BLAUNCH((kb_pjac<T, 3, 0>), kThreads, m, 0, ba);
                    }
            }
        }
        ISDC_BLAUNCH((kb_update<T>), kThreads, mupd[p], 0, A(o_upd[p], p, 0, 0));
    }
    for (int M = 1; M <= ISDC_MAX_M; ++M)
        if (mq[M].total) launch_quad_m<D>(M, mq[M], A(o_q[M], 0, 0, 0), s);
    ISDC_BLAUNCH(kb_reduce, kThreads, mred, 0, A(o_red, 0, 0, 0));
    };
    if (timing) {
        // measurement only: `reps` more sweeps of the running slots, eager or
        // replayed from one captured graph; no decisions, states unspecified
        hipEvent_t ev[2];
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        if (timing->graph) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            sweep();
            HIPCHK(hipStreamEndCapture(s, &g));
            HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            HIPCHK(hipGraphLaunch(ge, s));  // warm-up
            HIPCHK(hipEventRecord(ev[0], s));
            for (int r = 0; r < timing->reps; ++r) HIPCHK(hipGraphLaunch(ge, s));
            HIPCHK(hipEventRecord(ev[1], s));
            HIPCHK(hipStreamSynchronize(s));
            HIPCHK(hipGraphExecDestroy(ge));
            HIPCHK(hipGraphDestroy(g));
        } else {
            sweep();  // warm-up
            HIPCHK(hipEventRecord(ev[0], s));
            for (int r = 0; r < timing->reps; ++r) sweep();
            HIPCHK(hipEventRecord(ev[1], s));
            HIPCHK(hipStreamSynchronize(s));
        }
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev[0], ev[1]));
        timing->us = 1e3 * (double)ms / timing->reps;
        int launches = mred.total > 0;
        for (int M = 1; M <= ISDC_MAX_M; ++M) launches += mq[M].total > 0;
        for (int p = 0; p < maxns; ++p) {
            launches += (mrhs[p].total > 0) + (mupd[p].total > 0);
            int per_cycle = mtail[p].total > 0;
            for (int l = 0; l < maxlev; ++l) {
                per_cycle += 2 * (mlev[p][l].total > 0) + (D == 3 && mres[p][l].total > 0);
                for (int K = 1; K <= 3; ++K) per_cycle += (mjres[K][p][l].total > 0) + (mpjac[K][p][l].total > 0);
            }
            launches += L * per_cycle;
        }
        timing->launches = launches;
        for (auto& e : ev) (void)hipEventDestroy(e);
        return;
    }
    sweep();
    HIPCHK(hipMemcpyAsync(b->h_res, b->d_res, cap * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (FILE* trace = trace_stream()) {  // host time once the batch sweep's residuals are back
        const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now().time_since_epoch()).count();
        std::fprintf(trace, "isdc_trace batch=%p running=%d t_us=%.1f\n", (void*)b, (int)run.size(), us);
        std::fflush(trace);
    }
    // ---- decisions
    Map mend;
    for (int i : run) {
        Slot& sl = b->slots[i];
        const double res = b->h_res[i];
        sl.cur.sweeps += 1;
        sl.cur.vcycles += (int64_t)b->h_desc[i].ns * L;
        sl.cur.residual = res;
        if (sl.cur.hist_len < ISDC_HIST) sl.cur.residual_hist[sl.cur.hist_len++] = res;
        bool end_step = false;
        if (!std::isfinite(res)) {
            sl.status = ISDC_E_DIVERGED;
            end_step = true;
        } else if (res < sl.plan->par.sdc_tol) {
            end_step = true;
        } else if (sl.cur.sweeps >= sl.plan->par.max_sweeps) {
            sl.status = ISDC_E_NOT_CONVERGED;
            end_step = true;
        }
        if (end_step) {
            mend.add(i, ceil_div(b->h_desc[i].N, kChunkPts));
            sl.last = sl.cur;
            sl.vcycles_total += sl.cur.vcycles;
            std::memset(&sl.cur, 0, sizeof(sl.cur));
            sl.steps_done += 1;
            if (sl.status != ISDC_OK || sl.steps_done >= sl.nsteps) sl.state = SLOT_FINISHED;
            else sl.need_begin = true;
        } else {
            sl.parity ^= 1;
        }
    }
    if (mend.total) {
        // end copies read the buffer each ending slot wrote last
        SlotState* he = b->h_state[1];
        for (int i = 0; i < cap; ++i) he[i].parity = b->slots[i].parity;
        HIPCHK(hipMemcpyAsync(b->d_state, he, cap * sizeof(SlotState), hipMemcpyHostToDevice, s));
        MapBuf me{b};
        me.used = mb.used;
        const size_t o_end = me.put(mend);
        HIPCHK(hipMemcpyAsync(b->d_maps + o_end, b->h_maps + o_end, (me.used - o_end) * sizeof(int),
                              hipMemcpyHostToDevice, s));
        ISDC_BLAUNCH(kb_copy, kThreads, mend, 0, A(o_end, 0, 0, 1));
        // the staging buffers are reused by the next call: finish the copies first
        HIPCHK(hipStreamSynchronize(s));
    }
}

isdc_batch* as_batch(isdc_batch* b) {
    if (!b) fail(ISDC_E_INVAL, "batch is NULL");
    return b;
}

}  // namespace
}  // namespace isdc

using namespace isdc;

extern "C" {

int isdc_batch_workspace_bytes(int32_t capacity, size_t* out_bytes) {
    return guarded([&] {
        if (capacity < 1 || capacity > 4096) fail(ISDC_E_INVAL, "capacity must be in 1..4096");
        if (!out_bytes) fail(ISDC_E_INVAL, "out_bytes is NULL");
        *out_bytes = batch_layout(capacity, nullptr, nullptr);
    });
}

int isdc_batch_open(int32_t capacity, int32_t dim, int32_t precision, int32_t vcycles, void* d_workspace,
                    size_t bytes, isdc_batch** out) {
    return guarded([&] {
        if (capacity < 1 || capacity > 4096) fail(ISDC_E_INVAL, "capacity must be in 1..4096");
        if (dim < 1 || dim > 3) fail(ISDC_E_INVAL, "dim must be 1, 2 or 3");
        if (precision != ISDC_PREC_FP64 && precision != ISDC_PREC_MIXED) fail(ISDC_E_INVAL, "unknown precision");
        if (vcycles < 1 || vcycles > 64) fail(ISDC_E_INVAL, "batches need 1 <= vcycles <= 64");
        if (!out) fail(ISDC_E_INVAL, "out is NULL");
        *out = nullptr;
        const size_t need = batch_layout(capacity, nullptr, nullptr);
        if (!d_workspace || ((uintptr_t)d_workspace) % kAlign) fail(ISDC_E_WORKSPACE, "workspace NULL or misaligned");
        if (bytes < need) fail(ISDC_E_WORKSPACE, "batch workspace too small: need " + std::to_string(need));
        isdc_batch* b = new isdc_batch();
        b->cap = capacity;
        b->d = dim;
        b->prec = precision;
        b->L = vcycles;
        batch_layout(capacity, (char*)d_workspace, b);
        b->h_desc = nullptr;
        b->h_state[0] = b->h_state[1] = nullptr;
        b->h_res = nullptr;
        b->h_maps = nullptr;
        b->slots.assign(capacity, Slot());
        b->desc_dirty.assign(capacity, false);
        *out = b;
    });
}

int isdc_batch_bytes(int32_t count, const isdc_problem* probs, const isdc_params* pars, size_t* out_bytes) {
    return guarded([&] {
        if (count < 1 || count > 4096) fail(ISDC_E_INVAL, "count must be in 1..4096");
        if (!probs || !pars) fail(ISDC_E_INVAL, "NULL problems or params");
        if (!out_bytes) fail(ISDC_E_INVAL, "out_bytes is NULL");
        *out_bytes = fixed_layout(count, probs, pars, nullptr, nullptr);
    });
}

int isdc_batch_create(int32_t count, const isdc_problem* probs, const isdc_params* pars, void* d_workspace,
                      size_t bytes, isdc_batch** out) {
    return guarded([&] {
        if (count < 1 || count > 4096) fail(ISDC_E_INVAL, "count must be in 1..4096");
        if (!probs || !pars) fail(ISDC_E_INVAL, "NULL problems or params");
        if (!out) fail(ISDC_E_INVAL, "out is NULL");
        *out = nullptr;
        const size_t need = fixed_layout(count, probs, pars, nullptr, nullptr);
        if (!d_workspace || ((uintptr_t)d_workspace) % kAlign) fail(ISDC_E_WORKSPACE, "workspace NULL or misaligned");
        if (bytes < need) fail(ISDC_E_WORKSPACE, "batch workspace too small: need " + std::to_string(need));
        isdc_batch* b = nullptr;
        const int rc = isdc_batch_open(count, probs[0].dim, pars[0].precision, pars[0].vcycles, d_workspace,
                                       batch_layout(count, nullptr, nullptr), &b);
        if (rc != ISDC_OK) fail(rc, last_error());
        b->fixed = true;
        b->fprob.assign(probs, probs + count);
        b->fpar.assign(pars, pars + count);
        fixed_layout(count, probs, pars, (char*)d_workspace, b);
        *out = b;
    });
}

int isdc_batch_step(isdc_batch* b, double* const* d_u, const double* dt, const int32_t* active, void* stream,
                    isdc_stats* stats) {
    int status = ISDC_OK;
    int first_bad = -1;
    const int rc = guarded([&] {
        as_batch(b);
        if (!b->fixed) fail(ISDC_E_INVAL, "isdc_batch_step needs a batch made by isdc_batch_create");
        if (!d_u || !dt) fail(ISDC_E_INVAL, "NULL d_u or dt");
        for (int i = 0; i < b->cap; ++i)
            if (b->slots[i].state == SLOT_RUNNING) fail(ISDC_E_INVAL, "slots are running (isdc_batch_set use)");
        // validate every active instance before any device work
        int nact = 0;
        for (int i = 0; i < b->cap; ++i) {
            if (active && !active[i]) continue;
            if (!d_u[i]) fail(ISDC_E_INVAL, "d_u[" + std::to_string(i) + "] is NULL");
            if (!std::isfinite(dt[i]) || dt[i] <= 0) fail(ISDC_E_INVAL, "dt[" + std::to_string(i) + "] must be finite and > 0");
            ++nact;
        }
        for (int i = 0; i < b->cap; ++i) {
            if (active && !active[i]) continue;
            const int r = isdc_batch_set(b, i, &b->fprob[i], &b->fpar[i], b->fws[i], b->fbytes[i], d_u[i], dt[i], 1);
            if (r != ISDC_OK) fail(r, last_error());
        }
        int running = nact;
        while (running > 0) {
            const int r = isdc_batch_advance(b, stream, &running);
            if (r != ISDC_OK) fail(r, last_error());
        }
        for (int i = 0; i < b->cap; ++i) {
            if (active && !active[i]) continue;
            Slot& sl = b->slots[i];
            if (stats) stats[i] = sl.last;
            if (sl.status != ISDC_OK && status == ISDC_OK) {
                status = sl.status;
                first_bad = i;
            }
            sl.state = SLOT_FREE;  // the plan stays for the next step; the slot is ready to be set again
        }
    });
    if (rc != ISDC_OK) return rc;
    if (status != ISDC_OK)
        last_error() = std::string(status == ISDC_E_DIVERGED ? "non-finite SDC residual" : "SDC residual not below sdc_tol after max_sweeps") +
                       " in instance " + std::to_string(first_bad);
    return status;
}

void isdc_batch_destroy(isdc_batch* b) {
    if (!b) return;
    for (auto& sl : b->slots)
        if (sl.plan) isdc_destroy(sl.plan);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    for (int k = 0; k < 2; ++k)
        if (b->h_state[k]) (void)hipHostFree(b->h_state[k]);
    if (b->h_res) (void)hipHostFree(b->h_res);
    if (b->h_maps) (void)hipHostFree(b->h_maps);
    delete b;
}

int isdc_batch_set(isdc_batch* b, int32_t slot, const isdc_problem* prob, const isdc_params* par, void* d_plan_workspace,
                   size_t plan_bytes, double* d_u, double dt, int32_t nsteps) {
    return guarded([&] {
        as_batch(b);
        if (slot < 0 || slot >= b->cap) fail(ISDC_E_INVAL, "slot out of range");
        if (b->slots[slot].state == SLOT_RUNNING) fail(ISDC_E_INVAL, "slot is running");
        validate(prob, par);
        check_batch_params(b, prob, par);
        if (!d_u) fail(ISDC_E_INVAL, "d_u is NULL");
        if (!std::isfinite(dt) || dt <= 0) fail(ISDC_E_INVAL, "dt must be finite and > 0");
        if (nsteps < 1) fail(ISDC_E_INVAL, "nsteps must be >= 1");
        const size_t need = layout(*prob, *par, nullptr, nullptr);
        if (!d_plan_workspace || ((uintptr_t)d_plan_workspace) % kAlign)
            fail(ISDC_E_WORKSPACE, "slot workspace NULL or misaligned");
        if (plan_bytes < need) fail(ISDC_E_WORKSPACE, "slot workspace too small: need " + std::to_string(need));
        if (!b->h_desc) {  // pinned staging, allocated on first use
            void* ptr = nullptr;
            HIPCHK(hipHostMalloc(&ptr, (size_t)b->cap * sizeof(SlotDesc), hipHostMallocDefault));
            b->h_desc = (SlotDesc*)ptr;
            for (int k = 0; k < 2; ++k) {
                HIPCHK(hipHostMalloc(&ptr, (size_t)b->cap * sizeof(SlotState), hipHostMallocDefault));
                b->h_state[k] = (SlotState*)ptr;
                std::memset(ptr, 0, (size_t)b->cap * sizeof(SlotState));
            }
            HIPCHK(hipHostMalloc(&ptr, (size_t)b->cap * sizeof(double), hipHostMallocDefault));
            b->h_res = (double*)ptr;
            HIPCHK(hipHostMalloc(&ptr, b->maps_cap * sizeof(int), hipHostMallocDefault));
            b->h_maps = (int*)ptr;
        }
        Slot& sl = b->slots[slot];
        if (sl.plan) isdc_destroy(sl.plan);
        sl = Slot();
        sl.plan = new isdc_plan();
        init_plan(sl.plan, prob, par, d_plan_workspace);
        sl.state = SLOT_RUNNING;
        sl.u = d_u;
        sl.dt = dt;
        sl.nsteps = nsteps;
        sl.need_begin = true;
        build_desc(b, slot);
    });
}

int isdc_batch_advance(isdc_batch* b, void* stream, int32_t* h_running) {
    return guarded([&] {
        as_batch(b);
        std::vector<int> run;
        for (int i = 0; i < b->cap; ++i)
            if (b->slots[i].state == SLOT_RUNNING) run.push_back(i);
        if (!run.empty()) {
            hipStream_t s = (hipStream_t)stream;
            const int d = b->d;
            if (b->prec == ISDC_PREC_FP64) {
                if (d == 1) advance_impl<double, 1>(b, s, run);
                else if (d == 2) advance_impl<double, 2>(b, s, run);
                else advance_impl<double, 3>(b, s, run);
            } else {
                if (d == 1) advance_impl<float, 1>(b, s, run);
                else if (d == 2) advance_impl<float, 2>(b, s, run);
                else advance_impl<float, 3>(b, s, run);
            }
        }
        if (h_running) {
            int c = 0;
            for (auto& sl : b->slots) c += sl.state == SLOT_RUNNING;
            *h_running = c;
        }
    });
}

int isdc_batch_time_sweeps(isdc_batch* b, int32_t reps, int32_t graph, void* stream, double* h_us_per_sweep,
                           int32_t* h_launches) {
    return guarded([&] {
        as_batch(b);
        if (reps < 1 || reps > 10000) fail(ISDC_E_INVAL, "reps must be in 1..10000");
        if (graph != 0 && graph != 1) fail(ISDC_E_INVAL, "graph must be 0 or 1");
        if (!h_us_per_sweep) fail(ISDC_E_INVAL, "h_us_per_sweep is NULL");
        if (graph && !stream) fail(ISDC_E_INVAL, "graph capture needs a stream other than the null stream");
        std::vector<int> run;
        for (int i = 0; i < b->cap; ++i)
            if (b->slots[i].state == SLOT_RUNNING) {
                if (b->slots[i].need_begin) fail(ISDC_E_INVAL, "slots must have started their step (advance once first)");
                run.push_back(i);
            }
        if (run.empty()) fail(ISDC_E_INVAL, "no running slot");
        SweepTiming t{reps, graph != 0, 0.0, 0};
        hipStream_t s = (hipStream_t)stream;
        const int d = b->d;
        if (b->prec == ISDC_PREC_FP64) {
            if (d == 1) advance_impl<double, 1>(b, s, run, &t);
            else if (d == 2) advance_impl<double, 2>(b, s, run, &t);
            else advance_impl<double, 3>(b, s, run, &t);
        } else {
            if (d == 1) advance_impl<float, 1>(b, s, run, &t);
            else if (d == 2) advance_impl<float, 2>(b, s, run, &t);
            else advance_impl<float, 3>(b, s, run, &t);
        }
        *h_us_per_sweep = t.us;
        if (h_launches) *h_launches = t.launches;
    });
}

int isdc_batch_slot_info(const isdc_batch* b, int32_t slot, int32_t* state, int32_t* status, int32_t* steps_done,
                         isdc_stats* last_step) {
    return guarded([&] {
        if (!b) fail(ISDC_E_INVAL, "batch is NULL");
        if (slot < 0 || slot >= b->cap) fail(ISDC_E_INVAL, "slot out of range");
        const Slot& sl = b->slots[slot];
        if (state) *state = sl.state;
        if (status) *status = sl.status;
        if (steps_done) *steps_done = sl.steps_done;
        if (last_step) *last_step = sl.last;
    });
}

int isdc_batch_release(isdc_batch* b, int32_t slot) {
    return guarded([&] {
        as_batch(b);
        if (slot < 0 || slot >= b->cap) fail(ISDC_E_INVAL, "slot out of range");
        Slot& sl = b->slots[slot];
        if (sl.plan) isdc_destroy(sl.plan);
        sl = Slot();
    });
}

}  // extern "C"
