// Fourth-order compact stencil (Sec. 3, eq. (5)), 2D, with homogeneous
// Dirichlet or periodic boundaries, and the WENO5 advection of viscous
// Burgers (Sec. 4.1).
//
// The compact scheme carries a weighting matrix W = I + (h^2/12) L_h next to
// its 9-point Laplacian A_h = L_h + (h^2/6) D_x D_y:
//   A_h u = (4 (sum of the 4 edge neighbours) + (sum of the 4 corners) - 20 u) / (6 h^2)
//   W u   = u + (sum of the 4 edge neighbours - 4 u) / 12
// With f~(u) = W f^E(u) + nu A_h u the sweep of eq. (5) solves
//   (W - dt_m nu A_h) u_{m+1}^{k+1} = W [u_m^{k+1} + dt_m (f^E(u_m^{k+1}) - f^E(u_m^k))]
//                                     - dt_m nu A_h u_{m+1}^k + S_m F~(u^k),
// here in correction form from the guess g = u_{m+1}^k:
//   (W - c A_h) e = W [u_m^{k+1} - g + dt_m (f^E(u_m^{k+1}) - f^E(u_m^k))] + S_m F~,
// and the SDC residual is u_0 + W^{-1} (dt Q F~)_m - u_m, W inverted once per
// node.
//
// Multigrid for B_H = I + w L_H - c A_H (w = h^2/12 of the finest grid, so
// B_h = W - c A_h): weighted-Jacobi smoothing (red-black ordering is not a
// Gauss-Seidel sweep for a 9-point stencil), the residual fused with its full
// weighting, linear prolongation and a single-workgroup tail for the levels
// of at most 63^2 (Dirichlet) or 32^2 (periodic) points.  On a level with
// spacing H the stencil is
//   centre b0 = 1 - 4 w/H^2 + (10/3) c/H^2,  edges bf = w/H^2 - (2/3) c/H^2,
//   corners bc = -c / (6 H^2).
// Dirichlet grids have n = 2^k - 1 interior points per axis (coarse point I on
// fine point 2I+1, zero ghosts); periodic grids have n = 2^k points on
// [-1, 1) (coarse point I on fine point 2I, indices wrap, and on one point
// every neighbour is the point itself, so B_H = I there).
// These are the plain one-thread-per-point forms; the arrays stay in L2
// between neighbouring threads.
#include <hip/hip_runtime.h>

#include "ctail.h"
#include "internal.h"
#include "jrows.h"
#include "mg_device.h"
#include "sdc_device.h"
#include "tile_common.h"

namespace isdc {

namespace {

constexpr int kB = 256;

// u at (x, y); outside the grid zero (Dirichlet) or wrapped (periodic,
// offsets of at most n).
template <bool PER, typename T>
__device__ __forceinline__ T at(const T* __restrict__ u, int n, int x, int y) {
    if (PER) {
        x = x < 0 ? x + n : (x >= n ? x - n : x);
        y = y < 0 ? y + n : (y >= n ? y - n : y);
        return u[(size_t)y * n + x];
    }
    return ((unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n) ? u[(size_t)y * n + x] : T(0);
}

// Sums of the edge and of the corner neighbours.
template <bool PER, typename T>
__device__ __forceinline__ void nb9(const T* __restrict__ u, int n, int x, int y, T& edges, T& corners) {
    edges = at<PER>(u, n, x - 1, y) + at<PER>(u, n, x + 1, y) + at<PER>(u, n, x, y - 1) + at<PER>(u, n, x, y + 1);
    corners = at<PER>(u, n, x - 1, y - 1) + at<PER>(u, n, x + 1, y - 1) + at<PER>(u, n, x - 1, y + 1) +
              at<PER>(u, n, x + 1, y + 1);
}

template <bool PER, typename T>
__device__ __forceinline__ T apply_b(const T* __restrict__ u, int n, int x, int y, T uc, const CCoef<T>& k) {
    T edges, corners;
    nb9<PER>(u, n, x, y, edges, corners);
    return k.b0 * uc + k.bf * edges + k.bc * corners;
}

__device__ __forceinline__ double fe_of(double v, int fe) { return fe == ISDC_FE_CUBIC ? v - v * v * v : 0.0; }

template <typename T, bool ZERO, bool PER>
__global__ void __launch_bounds__(kB)
k_cjacobi(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, CCoef<T> k) {
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    const size_t i = (size_t)y * n + x;
    if (ZERO) {
        e_out[i] = k.omega * r[i] * k.inv_b0;
    } else {
        const T uc = e_in[i];
        e_out[i] = uc + k.omega * (r[i] - apply_b<PER>(e_in, n, x, y, uc, k)) * k.inv_b0;
    }
}

// K weighted-Jacobi steps in one launch on row-mapped tiles: a tile of
// (64 - 2K) x 16 points stages the iterate on the tile plus a halo of K in
// LDS (64 columns from x0 - K, one column per lane) and the right-hand side
// of its own points in registers, then runs step s on the tile plus a halo of
// K - s, ping-ponging between two LDS buffers; the last step leaves the tile.
// Each point is updated with the expression of k_cjacobi, so the result is
// that of K single-step launches.  Dirichlet: points outside the grid are
// zero and never updated; periodic: the staged box wraps, and points past
// the end of a ragged last tile repeat points of the first (same values),
// only the tile's own points are stored.
template <int K> struct JTile {
    static constexpr int TX = kJL - 2 * K, TY = kJTY;
    static constexpr int ROWS = TY + 2 * K;
    static constexpr int RP = kThreads / kJL;  // rows per block step
    static constexpr int IP = (ROWS + RP - 1) / RP;
    static constexpr int N = IP * kThreads;
};

template <typename T, bool PER, int K, bool ZERO, bool C9 = true>
__global__ void __launch_bounds__(kThreads)
k_cjacobi_k(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, int ntx, int nty,
            CCoef<T> k, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using J = JTile<K>;
    constexpr int L = kJL;
    __shared__ T sa[J::N];
    __shared__ T sb[J::N];
    int x0, y0, z0;
    tile_origin(ntx, nty, J::TX, J::TY, 1, x0, y0, z0);
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    // LDS column c is x = x0 - K + c, row q is y = y0 - K + q
    const int x = x0 - K + c;
    const int xg = PER ? (x < 0 ? x + n : (x >= n ? x - n : x)) : x;
    const bool xin = PER ? (c < J::TX + 2 * K) : (c < J::TX + 2 * K && x >= 0 && x < n);
    T vr[J::IP];
#pragma unroll
    for (int i = 0; i < J::IP; ++i) {
        const int q = j + i * J::RP;
        const int y = y0 - K + q;
        const int yg = PER ? (y < 0 ? y + n : (y >= n ? y - n : y)) : y;
        const bool in = xin && q < J::ROWS && (PER || (y >= 0 && y < n));
        T ve = T(0), rv = T(0);
        if (in) {
            const size_t gi = (size_t)yg * n + xg;
            if (!ZERO) ve = e_in[gi];
            rv = r[gi];
        }
        vr[i] = rv;
        sa[threadIdx.x + i * kThreads] = ve;
        sb[threadIdx.x + i * kThreads] = ve;
    }
    __syncthreads();
    // step s (1..K) updates the tile plus a halo of K - s: LDS columns and
    // rows s .. TX + 2K - 1 - s, inside the grid (Dirichlet)
    T* src = sa;
    T* dst = sb;
    const T w = k.omega, inv = k.inv_b0;
#pragma unroll
    for (int st = 1; st <= K; ++st) {
        const bool cok = c >= st && c <= J::TX + 2 * K - 1 - st && xin;
        T v[J::IP];
        bool wr[J::IP];
#pragma unroll
        for (int i = 0; i < J::IP; ++i) {
            const int q = j + i * J::RP;
            const int y = y0 - K + q;
            wr[i] = cok && q >= st && q <= J::TY + 2 * K - 1 - st && (PER || (y >= 0 && y < n));
            if (wr[i]) {
                const int a = threadIdx.x + i * kThreads;
                if (ZERO && st == 1) {
                    v[i] = w * vr[i] * inv;
                } else if (C9) {
                    const T uc = src[a];
                    const T edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                    const T corners = src[a - L - 1] + src[a - L + 1] + src[a + L - 1] + src[a + L + 1];
                    v[i] = uc + w * (vr[i] - (k.b0 * uc + k.bf * edges + k.bc * corners)) * inv;
                } else {
                    const T uc = src[a];
                    const T edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                    v[i] = uc + w * (vr[i] - (k.b0 * uc + k.bf * edges)) * inv;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < J::IP; ++i)
            if (wr[i]) dst[threadIdx.x + i * kThreads] = v[i];
        __syncthreads();
        T* t = src;
        src = dst;
        dst = t;
    }
    // the tile: columns / rows K .. K + T - 1, inside the grid
    if (c < K || c >= K + J::TX || x >= n || x < 0) return;
#pragma unroll
    for (int i = 0; i < J::IP; ++i) {
        const int q = j + i * J::RP;
        const int y = y0 - K + q;
        if (q >= K && q < K + J::TY && y < n) e_out[(size_t)y * n + x] = src[threadIdx.x + i * kThreads];
    }
}

template <typename T, bool PER, int K, bool ZERO, bool C9 = true>
__global__ void __launch_bounds__(kThreads)
k_cjres(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, T* __restrict__ rc, int n,
        int ntx, int nty, CCoef<T> k, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int x0, y0, z0;
    tile_origin(ntx, nty, CVT<K>::TX, CVT<K>::TY, 1, x0, y0, z0);
    cjres_tile<T, PER, K, ZERO, C9>(r, e_in, e_out, rc, n, x0, y0, k);
}

// MODE 0 writes the result to e_out; MODE 1 writes the float64 node value
// g + e to u_out instead (the last launch of an implicit solve).
template <typename T, bool PER, int K, bool C9 = true, int MODE = 0>
__global__ void __launch_bounds__(kThreads)
k_cpjac(const T* __restrict__ r, const T* __restrict__ e_in, const T* __restrict__ ec, T* __restrict__ e_out, int n,
        int ntx, int nty, CCoef<T> k, const double* __restrict__ g, double* __restrict__ u_out,
        const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int x0, y0, z0;
    tile_origin(ntx, nty, CVT<K>::TX, CVT<K>::TY, 1, x0, y0, z0);
    cpjac_tile<T, PER, K, C9, MODE>(r, e_in, ec, e_out, n, x0, y0, k, g, u_out);
}

// Residual r - B e on the fine points under each coarse point and its full
// weighting (1/4, 1/2, 1/4 per axis; coarse X sits on fine 2X+1, or on fine
// 2X with wrapped neighbours for periodic grids).
template <typename T, bool PER>
__global__ void __launch_bounds__(kB)
k_cresfw(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc, int n, CCoef<T> k) {
    const int nc = PER ? n / 2 : (n - 1) / 2;
    const int X = blockIdx.x * kB + threadIdx.x, Y = blockIdx.y;
    if (X >= nc) return;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        int y = PER ? 2 * Y + b - 1 : 2 * Y + b;
        if (PER) y = y < 0 ? y + n : y;
        T row = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int x = PER ? 2 * X + a - 1 : 2 * X + a;
            if (PER) x = x < 0 ? x + n : x;
            const size_t i = (size_t)y * n + x;
            row += w[a] * (r[i] - apply_b<PER>(e, n, x, y, e[i], k));
        }
        acc += w[b] * row;
    }
    rc[(size_t)Y * nc + X] = acc;
}

// Periodic linear interpolation added to u: fine 2I takes coarse I, fine
// 2I+1 the mean of coarse I and I+1 (wrapped), per axis.
template <typename T>
__global__ void __launch_bounds__(kB) k_cprolong_p(const T* __restrict__ ec, T* __restrict__ u, int n) {
    const int nc = n / 2;
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    const int X0 = x >> 1, Y0 = y >> 1;
    const int X1 = (x & 1) ? (X0 + 1 == nc ? 0 : X0 + 1) : X0;
    const int Y1 = (y & 1) ? (Y0 + 1 == nc ? 0 : Y0 + 1) : Y0;
    const T wx = (x & 1) ? T(0.5) : T(1), wy = (y & 1) ? T(0.5) : T(1);
    const T wx1 = (x & 1) ? T(0.5) : T(0), wy1 = (y & 1) ? T(0.5) : T(0);
    const T* r0 = ec + (size_t)Y0 * nc;
    const T* r1 = ec + (size_t)Y1 * nc;
    u[(size_t)y * n + x] += wy * (wx * r0[X0] + wx1 * r0[X1]) + wy1 * (wx * r1[X0] + wx1 * r1[X1]);
}

template <typename T, bool PER>
__global__ void __launch_bounds__(kB)
k_cresnorm(const T* __restrict__ r, const T* __restrict__ e, int n, CCoef<T> k, double* __restrict__ partial) {
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    double v = 0.0;
    if (x < n) {
        const size_t i = (size_t)y * n + x;
        v = fabs((double)(r[i] - apply_b<PER>(e, n, x, y, e[i], k)));
    }
    v = block_max(v);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// r = W base + SF_m, base = u_m^{k+1} - u_{m+1}^k + dt_m (f^E(u_m^{k+1}) - f^E(u_m^k)),
// f^E pointwise or from the node arrays fe_new / fe_old.
template <typename T, bool PER>
__global__ void __launch_bounds__(kB) k_crhs(CRhsArgs a, T* __restrict__ out) {
    const int n = a.n;
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    auto base = [&](int xx, int yy) -> double {
        if (PER) {
            xx = xx < 0 ? xx + n : (xx >= n ? xx - n : xx);
            yy = yy < 0 ? yy + n : (yy >= n ? yy - n : yy);
        } else if ((unsigned)xx >= (unsigned)n || (unsigned)yy >= (unsigned)n) {
            return 0.0;
        }
        const size_t j = (size_t)yy * n + xx;
        const double un = a.um_new[j];
        // u_m^k only enters through f^E: not read for f^E = 0
        const double dfe = a.fe_new ? a.fe_new[j] - a.fe_old[j]
                                    : fe_of(un, a.fe) - fe_of(a.fe == ISDC_FE_ZERO ? 0.0 : a.um_old[j], a.fe);
        return un - a.up_old[j] + a.dtm * dfe;
    };
    const double bc = base(x, y);
    const double edges = base(x - 1, y) + base(x + 1, y) + base(x, y - 1) + base(x, y + 1);
    const size_t i = (size_t)y * n + x;
    out[i] = T(bc + (edges - 4.0 * bc) / 12.0 + a.sf[i]);
}

// f~_j = W f^E(u_j) + nu A_h u_j at every node; SF_m = sum_j dt s_{m,j} f~_j
// and Y_m = sum_j dt q_{m,j} f~_j (the residual's right-hand side before W^{-1}).
template <int M, bool PER>
__global__ void __launch_bounds__(kB) k_cquad(CQuadArgs a) {
    const int n = a.n;
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    const size_t i = (size_t)y * n + x;
    double sf[M], yq[M];
#pragma unroll
    for (int m = 0; m < M; ++m) sf[m] = yq[m] = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double* u = a.u[j + 1];
        const double uc = u[i];
        double edges, corners;
        nb9<PER>(u, n, x, y, edges, corners);
        double fec, fe_edges;
        if (a.feu[j + 1]) {
            const double* g = a.feu[j + 1];
            fec = g[i];
            fe_edges = at<PER>(g, n, x - 1, y) + at<PER>(g, n, x + 1, y) + at<PER>(g, n, x, y - 1) +
                       at<PER>(g, n, x, y + 1);
        } else {
            fec = fe_of(uc, a.fe);
            fe_edges = 0.0;
            if (a.fe == ISDC_FE_CUBIC)
                fe_edges = fe_of(at<PER>(u, n, x - 1, y), a.fe) + fe_of(at<PER>(u, n, x + 1, y), a.fe) +
                           fe_of(at<PER>(u, n, x, y - 1), a.fe) + fe_of(at<PER>(u, n, x, y + 1), a.fe);
        }
        const double f = fec + (fe_edges - 4.0 * fec) / 12.0 + a.nu_6h2 * (4.0 * edges + corners - 20.0 * uc);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            sf[m] += a.dtS[m * ISDC_MAX_M + j] * f;
            yq[m] += a.dtQ[m * ISDC_MAX_M + j] * f;
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        if (a.sf[m]) a.sf[m][i] = sf[m];
        if (a.y[m]) a.y[m][i] = yq[m];
    }
}

// Per-node partial maxima of |u_0 + x_m - u_m| (x_m = W^{-1} Y_m): block
// (b, k) covers a stride of node k's points.
__global__ void __launch_bounds__(kB) k_cres(CResArgs a, double* __restrict__ partial) {
    const int k = blockIdx.y;
    const double* um = a.um[k];
    const double* xm = a.xm[k];
    double v = 0.0;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < a.N; i += (size_t)gridDim.x * kB)
        v = nanmax(v, fabs(a.u0[i] + xm[i] - um[i]));
    v = block_max(v);
    if (threadIdx.x == 0) partial[(size_t)k * gridDim.x + blockIdx.x] = v;
}

// ---------------------------------------------------------------- W^{-1} by Chebyshev iteration
// W = I + (h^2/12) L_h on the finest grid: W x = x + (edges - 4 x) / 12, whose
// Jacobi-scaled spectrum D^{-1} W lies in [1/2, 3/2] (D = 2/3) for both
// boundary conditions.  One step of the Chebyshev iteration on that interval
// (centre 1, half-width 1/2):
//   r = D^{-1} (y - W x),  d = cd d + cr r  (first step: d = r),  x_out = x + d.
// KIND 0: first step from x = 0 (x_in not read); 1: first step from x_in;
// 2: a later step.
constexpr double kTwelfth = 1.0 / 12.0;
template <bool PER, int KIND>
__global__ void __launch_bounds__(kB)
k_wcheb(const double* __restrict__ y, const double* __restrict__ x_in, double* __restrict__ x_out,
        double* __restrict__ d, int n, double cd, double cr) {
    const int x = blockIdx.x * kB + threadIdx.x, yy = blockIdx.y;
    if (x >= n) return;
    const size_t i = (size_t)yy * n + x;
    double wx = 0.0;
    if (KIND != 0) {
        const double c = x_in[i];
        const double edges = at<PER>(x_in, n, x - 1, yy) + at<PER>(x_in, n, x + 1, yy) + at<PER>(x_in, n, x, yy - 1) +
                             at<PER>(x_in, n, x, yy + 1);
        wx = c + (edges - 4.0 * c) * kTwelfth;
    }
    const double r = (y[i] - wx) * 1.5;
    const double dn = KIND == 2 ? cd * d[i] + cr * r : r;
    d[i] = dn;
    x_out[i] = (KIND != 0 ? x_in[i] : 0.0) + dn;
}

// kWS consecutive Chebyshev steps in one launch on the row-mapped tiles of
// the Jacobi kernel above: x on the tile plus a halo of kWS in LDS (two
// buffers), y and d of the thread's points in registers; step s runs on the
// tile plus a halo of kWS - s with its own coefficients (cd[s], cr[s]).  Every
// point is updated with the expression of k_wcheb, so the result is that of
// kWS single steps.  KIND: the first step's kind as in k_wcheb.  d is read on
// the halo, so it goes from d_in to d_out (x from x_in to x_out).
constexpr int kWS = 4;
struct WChebCoefs {
    double cd[kWS], cr[kWS];
};

template <bool PER, int KIND>
__global__ void __launch_bounds__(kThreads)
k_wcheb_k(const double* __restrict__ y, const double* __restrict__ x_in, double* __restrict__ x_out,
          const double* __restrict__ d_in, double* __restrict__ d_out, int n, int ntx, int nty, WChebCoefs co) {
    using J = JTile<kWS>;
    constexpr int K = kWS, L = kJL;
    __shared__ double sa[J::N];
    __shared__ double sb[J::N];
    int x0, y0, z0;
    tile_origin(ntx, nty, J::TX, J::TY, 1, x0, y0, z0);
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    const int x = x0 - K + c;
    const int xg = PER ? (x < 0 ? x + n : (x >= n ? x - n : x)) : x;
    const bool xin = PER ? true : (x >= 0 && x < n);
    double vy[J::IP], vd[J::IP];
#pragma unroll
    for (int i = 0; i < J::IP; ++i) {
        const int q = j + i * J::RP;
        const int yy = y0 - K + q;
        const int yg = PER ? (yy < 0 ? yy + n : (yy >= n ? yy - n : yy)) : yy;
        const bool in = xin && q < J::ROWS && (PER || (yy >= 0 && yy < n));
        double vx = 0.0, a = 0.0, b = 0.0;
        if (in) {
            const size_t gi = (size_t)yg * n + xg;
            if (KIND != 0) vx = x_in[gi];
            a = y[gi];
            if (KIND == 2) b = d_in[gi];
        }
        vy[i] = a;
        vd[i] = b;
        sa[threadIdx.x + i * kThreads] = vx;
        sb[threadIdx.x + i * kThreads] = vx;
    }
    __syncthreads();
    double* src = sa;
    double* dst = sb;
#pragma unroll
    for (int st = 1; st <= K; ++st) {
        const bool first = st == 1;
        const bool cok = c >= st && c <= J::TX + 2 * K - 1 - st && xin;
        double v[J::IP];
        bool wr[J::IP];
#pragma unroll
        for (int i = 0; i < J::IP; ++i) {
            const int q = j + i * J::RP;
            const int yy = y0 - K + q;
            wr[i] = cok && q >= st && q <= J::TY + 2 * K - 1 - st && (PER || (yy >= 0 && yy < n));
            if (wr[i]) {
                const int a = threadIdx.x + i * kThreads;
                double wx = 0.0, xc = 0.0;
                if (!(first && KIND == 0)) {
                    xc = src[a];
                    const double edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                    wx = xc + (edges - 4.0 * xc) * kTwelfth;
                }
                const double r = (vy[i] - wx) * 1.5;
                const double dn = (first && KIND != 2) ? r : co.cd[st - 1] * vd[i] + co.cr[st - 1] * r;
                vd[i] = dn;
                v[i] = xc + dn;
            }
        }
#pragma unroll
        for (int i = 0; i < J::IP; ++i)
            if (wr[i]) dst[threadIdx.x + i * kThreads] = v[i];
        __syncthreads();
        double* t = src;
        src = dst;
        dst = t;
    }
    if (c < K || c >= K + J::TX || x >= n || x < 0) return;
#pragma unroll
    for (int i = 0; i < J::IP; ++i) {
        const int q = j + i * J::RP;
        const int yy = y0 - K + q;
        if (q >= K && q < K + J::TY && yy < n) {
            const size_t gi = (size_t)yy * n + x;
            x_out[gi] = src[threadIdx.x + i * kThreads];
            d_out[gi] = vd[i];
        }
    }
}

// ---------------------------------------------------------------- WENO5 advection
// f^E(u) = -sum over axes of (F_{i+1/2} - F_{i-1/2}) / h for the flux u^2/2
// (periodic).  F_{i+1/2} is the fifth-order WENO reconstruction (Jiang-Shu
// smoothness indicators and linear weights 1/10, 6/10, 3/10, epsilon 1e-6) of
// the split fluxes (u^2/2 +/- alpha u) / 2, alpha = max(|u_i|, |u_{i+1}|):
// the + part from u_{i-2..i+2}, the - part mirrored from u_{i+3..i-1}.

__device__ __forceinline__ double weno5_face(double a, double b, double c, double d, double e) {
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0;
    const double q1 = (-b + 5.0 * c + 2.0 * d) / 6.0;
    const double q2 = (2.0 * c + 5.0 * d - e) / 6.0;
    const double t0 = a - 2.0 * b + c, s0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, s1 = b - d;
    const double t2 = c - 2.0 * d + e, s2 = 3.0 * c - 4.0 * d + e;
    const double b0 = 13.0 / 12.0 * t0 * t0 + 0.25 * s0 * s0;
    const double b1 = 13.0 / 12.0 * t1 * t1 + 0.25 * s1 * s1;
    const double b2 = 13.0 / 12.0 * t2 * t2 + 0.25 * s2 * s2;
    const double eps = 1e-6;
    const double a0 = 0.1 / ((eps + b0) * (eps + b0));
    const double a1 = 0.6 / ((eps + b1) * (eps + b1));
    const double a2 = 0.3 / ((eps + b2) * (eps + b2));
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// Flux at the face between v[2] and v[3] from v[0..5] = u_{i-2..i+3}.
__device__ __forceinline__ double weno5_flux(const double* v) {
    const double alpha = fmax(fabs(v[2]), fabs(v[3]));
    double fp[6], fm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double f = 0.5 * v[k] * v[k];
        fp[k] = 0.5 * (f + alpha * v[k]);
        fm[k] = 0.5 * (f - alpha * v[k]);
    }
    return weno5_face(fp[0], fp[1], fp[2], fp[3], fp[4]) + weno5_face(fm[5], fm[4], fm[3], fm[2], fm[1]);
}

__global__ void __launch_bounds__(kB) k_weno_burgers(const double* __restrict__ u, double* __restrict__ out, int n,
                                                    double inv_h) {
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    double vx[7], vy[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        vx[k] = at<true>(u, n, x + k - 3, y);
        vy[k] = at<true>(u, n, x, y + k - 3);
    }
    const double dy = weno5_flux(vy + 1) - weno5_flux(vy);
    const double dx = weno5_flux(vx + 1) - weno5_flux(vx);
    out[(size_t)y * n + x] = -(dy * inv_h) - dx * inv_h;
}

// ---------------------------------------------------------------- compact tail
// One V-cycle of B on levels n_t, ..., 1 in one workgroup (ctail.h).

template <typename T, bool PER>
__global__ void __launch_bounds__(kTail)
k_ctail(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t, CTailCoefs tc, int nu1, int nu2, double omega,
        int zero_guess) {
    ctail_body<T, PER>(rhs_g, e_g, n_t, tc, nu1, nu2, omega, zero_guess);
}

dim3 grid2(int n) { return dim3((n + kB - 1) / kB, n); }

}  // namespace

template <typename T>
CCoef<T> make_ccoef(double c, double w, double H, double omega) {
    const double iH2 = 1.0 / (H * H);
    CCoef<T> k;
    const double b0 = 1.0 - 4.0 * w * iH2 + (10.0 / 3.0) * c * iH2;
    k.b0 = T(b0);
    k.bf = T(w * iH2 - (2.0 / 3.0) * c * iH2);
    k.bc = T(-c * iH2 / 6.0);
    k.inv_b0 = T(1.0 / b0);
    k.omega = T(omega);
    return k;
}

template <typename T>
CCoef<T> make_coef5(double c, double h, double omega) {
    const double a = c / (h * h);
    const double b0 = 1.0 + 4.0 * a;
    CCoef<T> k;
    k.b0 = T(b0);
    k.bf = T(-a);
    k.bc = T(0);
    k.inv_b0 = T(1.0 / b0);
    k.omega = T(omega);
    return k;
}

template <typename T>
hipError_t launch_cjacobi(int n, const CCoef<T>& k, bool zero, const T* r, const T* e_in, T* e_out, bool per,
                          hipStream_t s) {
    if (per) {
        if (zero)
            hipLaunchKernelGGL((k_cjacobi<T, true, true>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
        else
            hipLaunchKernelGGL((k_cjacobi<T, false, true>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
    } else {
        if (zero)
            hipLaunchKernelGGL((k_cjacobi<T, true, false>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
        else
            hipLaunchKernelGGL((k_cjacobi<T, false, false>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cjacobi_steps(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out,
                                bool per, hipStream_t s) {
    if (nsteps == 1) return launch_cjacobi<T>(n, k, zero, r, e_in, e_out, per, s);
#define ISDC_CJK(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, JTile<KV>::TX, JTile<KV>::TY, 1, ntx, nty, nb);                                     \
        if (per && zero) ISDC_GLAUNCH((k_cjacobi_k<T, true, KV, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
        else if (per) ISDC_GLAUNCH((k_cjacobi_k<T, true, KV, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
        else if (zero) ISDC_GLAUNCH((k_cjacobi_k<T, false, KV, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
        else ISDC_GLAUNCH((k_cjacobi_k<T, false, KV, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
    }
    if (nsteps == 2) ISDC_CJK(2)
    else if (nsteps == 3) ISDC_CJK(3)
    else return hipErrorInvalidValue;
#undef ISDC_CJK
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cjres(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out, T* rc,
                        bool per, hipStream_t s) {
#define ISDC_CJR(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, CVT<KV>::TX, CVT<KV>::TY, 1, ntx, nty, nb);                                         \
        if (per && zero) ISDC_GLAUNCH((k_cjres<T, true, KV, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
        else if (per) ISDC_GLAUNCH((k_cjres<T, true, KV, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
        else if (zero) ISDC_GLAUNCH((k_cjres<T, false, KV, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
        else ISDC_GLAUNCH((k_cjres<T, false, KV, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
    }
    if (nsteps == 1) ISDC_CJR(1)
    else if (nsteps == 2) ISDC_CJR(2)
    else if (nsteps == 3) ISDC_CJR(3)
    else return hipErrorInvalidValue;
#undef ISDC_CJR
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cpjac(int n, const CCoef<T>& k, int nsteps, const T* r, const T* e_in, const T* ec, T* e_out,
                        bool per, hipStream_t s) {
#define ISDC_CPJ(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, CVT<KV>::TX, CVT<KV>::TY, 1, ntx, nty, nb);                                         \
        if (per) ISDC_GLAUNCH((k_cpjac<T, true, KV>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, k, nullptr, nullptr); \
        else ISDC_GLAUNCH((k_cpjac<T, false, KV>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, k, nullptr, nullptr); \
    }
    if (nsteps == 1) ISDC_CPJ(1)
    else if (nsteps == 2) ISDC_CPJ(2)
    else if (nsteps == 3) ISDC_CPJ(3)
    else return hipErrorInvalidValue;
#undef ISDC_CPJ
    return hipGetLastError();
}

// The same fused kernels for the second-order five-point operator
// A = I - c L_h (Dirichlet): b0 = 1 + 4a, bf = -a, no corner term.
template <typename T>
hipError_t launch_jacobi5_steps(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out,
                                hipStream_t s) {
#define ISDC_J5K(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, JTile<KV>::TX, JTile<KV>::TY, 1, ntx, nty, nb);                                     \
        if (zero) ISDC_GLAUNCH((k_cjacobi_k<T, false, KV, true, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
        else ISDC_GLAUNCH((k_cjacobi_k<T, false, KV, false, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, k); \
    }
    if (nsteps == 1) ISDC_J5K(1)
    else if (nsteps == 2) ISDC_J5K(2)
    else if (nsteps == 3) ISDC_J5K(3)
    else return hipErrorInvalidValue;
#undef ISDC_J5K
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jres5(int n, const CCoef<T>& k, int nsteps, bool zero, const T* r, const T* e_in, T* e_out, T* rc,
                        hipStream_t s) {
#define ISDC_J5R(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, CVT<KV>::TX, CVT<KV>::TY, 1, ntx, nty, nb);                                         \
        if (zero) ISDC_GLAUNCH((k_cjres<T, false, KV, true, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
        else ISDC_GLAUNCH((k_cjres<T, false, KV, false, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, k); \
    }
    if (nsteps == 1) ISDC_J5R(1)
    else if (nsteps == 2) ISDC_J5R(2)
    else if (nsteps == 3) ISDC_J5R(3)
    else return hipErrorInvalidValue;
#undef ISDC_J5R
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pjac5(int n, const CCoef<T>& k, int nsteps, const T* r, const T* e_in, const T* ec, T* e_out,
                        const double* g, double* u_out, hipStream_t s) {
#define ISDC_P5J(KV)                                                                                          \
    {                                                                                                         \
        int ntx, nty, nb;                                                                                     \
        tile_counts<2>(n, CVT<KV>::TX, CVT<KV>::TY, 1, ntx, nty, nb);                                         \
        if (u_out) ISDC_GLAUNCH((k_cpjac<T, false, KV, false, 1>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, k, g, u_out); \
        else ISDC_GLAUNCH((k_cpjac<T, false, KV, false, 0>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, k, nullptr, nullptr); \
    }
    if (nsteps == 1) ISDC_P5J(1)
    else if (nsteps == 2) ISDC_P5J(2)
    else if (nsteps == 3) ISDC_P5J(3)
    else return hipErrorInvalidValue;
#undef ISDC_P5J
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cresfw(int n, const CCoef<T>& k, const T* r, const T* e, T* rc, bool per, hipStream_t s) {
    if (per)
        hipLaunchKernelGGL((k_cresfw<T, true>), grid2(n / 2), dim3(kB), 0, s, r, e, rc, n, k);
    else
        hipLaunchKernelGGL((k_cresfw<T, false>), grid2((n - 1) / 2), dim3(kB), 0, s, r, e, rc, n, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cprolong_p(int n, const T* ec, T* u, hipStream_t s) {
    hipLaunchKernelGGL((k_cprolong_p<T>), grid2(n), dim3(kB), 0, s, ec, u, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cresnorm(int n, const CCoef<T>& k, const T* r, const T* e, double* partial, int* nblocks, bool per,
                           hipStream_t s) {
    const dim3 g = grid2(n);
    *nblocks = (int)(g.x * g.y);
    if (per)
        hipLaunchKernelGGL((k_cresnorm<T, true>), g, dim3(kB), 0, s, r, e, n, k, partial);
    else
        hipLaunchKernelGGL((k_cresnorm<T, false>), g, dim3(kB), 0, s, r, e, n, k, partial);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_crhs(const CRhsArgs& a, T* out, bool per, hipStream_t s) {
    if (per)
        hipLaunchKernelGGL((k_crhs<T, true>), grid2(a.n), dim3(kB), 0, s, a, out);
    else
        hipLaunchKernelGGL((k_crhs<T, false>), grid2(a.n), dim3(kB), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_cquad(const CQuadArgs& a, int M, bool per, hipStream_t s) {
    switch (M) {
#define ISDC_CQ(MM)                                                                          \
    case MM:                                                                                 \
        if (per) hipLaunchKernelGGL((k_cquad<MM, true>), grid2(a.n), dim3(kB), 0, s, a);      \
        else hipLaunchKernelGGL((k_cquad<MM, false>), grid2(a.n), dim3(kB), 0, s, a);         \
        break;
        ISDC_CQ(1) ISDC_CQ(2) ISDC_CQ(3) ISDC_CQ(4) ISDC_CQ(5) ISDC_CQ(6) ISDC_CQ(7) ISDC_CQ(8) ISDC_CQ(9)
#undef ISDC_CQ
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cres(const CResArgs& a, double* partial, int* nblocks, hipStream_t s) {
    const int per = kCResBlocks;
    *nblocks = per * a.count;
    hipLaunchKernelGGL(k_cres, dim3(per, a.count), dim3(kB), 0, s, a, partial);
    return hipGetLastError();
}

hipError_t launch_wcheb(int n, bool per, int kind, const double* y, const double* x_in, double* x_out, double* d,
                        double cd, double cr, hipStream_t s) {
#define ISDC_WCHEB(P, K) \
    hipLaunchKernelGGL((k_wcheb<P, K>), grid2(n), dim3(kB), 0, s, y, x_in, x_out, d, n, cd, cr)
    if (per) {
        if (kind == 0) ISDC_WCHEB(true, 0); else if (kind == 1) ISDC_WCHEB(true, 1); else ISDC_WCHEB(true, 2);
    } else {
        if (kind == 0) ISDC_WCHEB(false, 0); else if (kind == 1) ISDC_WCHEB(false, 1); else ISDC_WCHEB(false, 2);
    }
#undef ISDC_WCHEB
    return hipGetLastError();
}

hipError_t launch_wcheb_steps(int n, bool per, int kind, int nsteps, const double* y, const double* x_in,
                              double* x_out, const double* d_in, double* d_out, const double* cd, const double* cr,
                              hipStream_t s) {
    if (nsteps != kWS) return hipErrorInvalidValue;
    WChebCoefs co;
    for (int k = 0; k < kWS; ++k) {
        co.cd[k] = cd[k];
        co.cr[k] = cr[k];
    }
    int ntx, nty, nb;
    tile_counts<2>(n, JTile<kWS>::TX, JTile<kWS>::TY, 1, ntx, nty, nb);
#define ISDC_WCHK(P, K) \
    hipLaunchKernelGGL((k_wcheb_k<P, K>), dim3(nb), dim3(kThreads), 0, s, y, x_in, x_out, d_in, d_out, n, ntx, nty, co)
    if (per) {
        if (kind == 0) ISDC_WCHK(true, 0); else if (kind == 1) ISDC_WCHK(true, 1); else ISDC_WCHK(true, 2);
    } else {
        if (kind == 0) ISDC_WCHK(false, 0); else if (kind == 1) ISDC_WCHK(false, 1); else ISDC_WCHK(false, 2);
    }
#undef ISDC_WCHK
    return hipGetLastError();
}

hipError_t launch_weno_burgers(int n, double h, const double* u, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_weno_burgers, grid2(n), dim3(kB), 0, s, u, out, n, 1.0 / h);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ctail(const MGConfig& mg, int n, double c, double w, double h, bool zero, const T* rhs, T* e,
                        bool per, hipStream_t s) {
    // Dirichlet n = 2^k - 1 <= 63, periodic n = 2^k <= 32
    const bool ok = per ? (n >= 1 && n <= kCTailMaxPeriodic && (n & (n - 1)) == 0)
                        : (n >= 1 && n <= kCTailMaxDirichlet && ((n + 1) & n) == 0);
    if (!ok) return hipErrorInvalidValue;
    CTailCoefs tc;
    double H = h;
    for (int l = 0; l < 16; ++l) {
        const CCoef<double> k = make_ccoef<double>(c, w, H, 1.0);
        tc.b0[l] = k.b0;
        tc.bf[l] = k.bf;
        tc.bc[l] = k.bc;
        H *= 2.0;
    }
    if (per)
        hipLaunchKernelGGL((k_ctail<T, true>), dim3(1), dim3(kTail), 0, s, rhs, e, n, tc, mg.nu_pre, mg.nu_post,
                           mg.omega, zero ? 1 : 0);
    else
        hipLaunchKernelGGL((k_ctail<T, false>), dim3(1), dim3(kTail), 0, s, rhs, e, n, tc, mg.nu_pre, mg.nu_post,
                           mg.omega, zero ? 1 : 0);
    return hipGetLastError();
}

#define ISDC_CINST(T)                                                                                              \
    template CCoef<T> make_ccoef<T>(double, double, double, double);                                               \
    template CCoef<T> make_coef5<T>(double, double, double);                                                       \
    template hipError_t launch_cjacobi<T>(int, const CCoef<T>&, bool, const T*, const T*, T*, bool, hipStream_t);   \
    template hipError_t launch_cjacobi_steps<T>(int, const CCoef<T>&, int, bool, const T*, const T*, T*, bool,      \
                                                hipStream_t);                                                      \
    template hipError_t launch_cjres<T>(int, const CCoef<T>&, int, bool, const T*, const T*, T*, T*, bool,          \
                                        hipStream_t);                                                              \
    template hipError_t launch_cpjac<T>(int, const CCoef<T>&, int, const T*, const T*, const T*, T*, bool,          \
                                        hipStream_t);                                                              \
    template hipError_t launch_cresfw<T>(int, const CCoef<T>&, const T*, const T*, T*, bool, hipStream_t);          \
    template hipError_t launch_jacobi5_steps<T>(int, const CCoef<T>&, int, bool, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_jres5<T>(int, const CCoef<T>&, int, bool, const T*, const T*, T*, T*, hipStream_t);  \
    template hipError_t launch_pjac5<T>(int, const CCoef<T>&, int, const T*, const T*, const T*, T*, const double*, \
                                        double*, hipStream_t);                                                     \
    template hipError_t launch_cprolong_p<T>(int, const T*, T*, hipStream_t);                                       \
    template hipError_t launch_cresnorm<T>(int, const CCoef<T>&, const T*, const T*, double*, int*, bool, hipStream_t); \
    template hipError_t launch_crhs<T>(const CRhsArgs&, T*, bool, hipStream_t);                                    \
    template hipError_t launch_ctail<T>(const MGConfig&, int, double, double, double, bool, const T*, T*, bool,     \
                                        hipStream_t);
ISDC_CINST(float)
ISDC_CINST(double)
#undef ISDC_CINST

}  // namespace isdc
