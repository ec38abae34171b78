// Fourth-order compact stencil (Sec. 3, eq. (5)), 2D.
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
// weighting, linear prolongation (the plain kernel), and a single-workgroup
// tail for the levels of 63^2 points and fewer.  On a level with spacing H the stencil is
//   centre b0 = 1 - 4 w/H^2 + (10/3) c/H^2,  edges bf = w/H^2 - (2/3) c/H^2,
//   corners bc = -c / (6 H^2).
// These are the plain one-thread-per-point forms; the arrays stay in L2
// between neighbouring threads.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mg_device.h"
#include "sdc_device.h"

namespace isdc {

namespace {

constexpr int kB = 256;

template <typename T>
__device__ __forceinline__ T at(const T* __restrict__ u, int n, int x, int y) {
    return ((unsigned)x < (unsigned)n && (unsigned)y < (unsigned)n) ? u[(size_t)y * n + x] : T(0);
}

// Sums of the edge and of the corner neighbours (zero ghosts).
template <typename T>
__device__ __forceinline__ void nb9(const T* __restrict__ u, int n, int x, int y, T& edges, T& corners) {
    edges = at(u, n, x - 1, y) + at(u, n, x + 1, y) + at(u, n, x, y - 1) + at(u, n, x, y + 1);
    corners = at(u, n, x - 1, y - 1) + at(u, n, x + 1, y - 1) + at(u, n, x - 1, y + 1) + at(u, n, x + 1, y + 1);
}

template <typename T>
__device__ __forceinline__ T apply_b(const T* __restrict__ u, int n, int x, int y, T uc, const CCoef<T>& k) {
    T edges, corners;
    nb9(u, n, x, y, edges, corners);
    return k.b0 * uc + k.bf * edges + k.bc * corners;
}

__device__ __forceinline__ double fe_of(double v, int fe) { return fe == ISDC_FE_CUBIC ? v - v * v * v : 0.0; }

template <typename T, bool ZERO>
__global__ void __launch_bounds__(kB)
k_cjacobi(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, CCoef<T> k) {
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    const size_t i = (size_t)y * n + x;
    if (ZERO) {
        e_out[i] = k.omega * r[i] * k.inv_b0;
    } else {
        const T uc = e_in[i];
        e_out[i] = uc + k.omega * (r[i] - apply_b(e_in, n, x, y, uc, k)) * k.inv_b0;
    }
}

// Residual r - B e on the fine points under each coarse point and its full
// weighting (1/4, 1/2, 1/4 per axis; fine index 2X+1 sits on coarse X).
template <typename T>
__global__ void __launch_bounds__(kB)
k_cresfw(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc, int n, CCoef<T> k) {
    const int nc = (n - 1) / 2;
    const int X = blockIdx.x * kB + threadIdx.x, Y = blockIdx.y;
    if (X >= nc) return;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int y = 2 * Y + b;
        T row = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int x = 2 * X + a;
            const size_t i = (size_t)y * n + x;
            row += w[a] * (r[i] - apply_b(e, n, x, y, e[i], k));
        }
        acc += w[b] * row;
    }
    rc[(size_t)Y * nc + X] = acc;
}

template <typename T>
__global__ void __launch_bounds__(kB)
k_cresnorm(const T* __restrict__ r, const T* __restrict__ e, int n, CCoef<T> k, double* __restrict__ partial) {
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    double v = 0.0;
    if (x < n) {
        const size_t i = (size_t)y * n + x;
        v = fabs((double)(r[i] - apply_b(e, n, x, y, e[i], k)));
    }
    v = block_max(v);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = v;
}

// r = W base + SF_m, base = u_m^{k+1} - u_{m+1}^k + dt_m (f^E(u_m^{k+1}) - f^E(u_m^k)).
template <typename T>
__global__ void __launch_bounds__(kB) k_crhs(CRhsArgs a, T* __restrict__ out) {
    const int n = a.n;
    const int x = blockIdx.x * kB + threadIdx.x, y = blockIdx.y;
    if (x >= n) return;
    auto base = [&](int xx, int yy) -> double {
        if ((unsigned)xx >= (unsigned)n || (unsigned)yy >= (unsigned)n) return 0.0;
        const size_t j = (size_t)yy * n + xx;
        const double un = a.um_new[j], uo = a.um_old[j];
        return un - a.up_old[j] + a.dtm * (fe_of(un, a.fe) - fe_of(uo, a.fe));
    };
    const double bc = base(x, y);
    const double edges = base(x - 1, y) + base(x + 1, y) + base(x, y - 1) + base(x, y + 1);
    const size_t i = (size_t)y * n + x;
    out[i] = T(bc + (edges - 4.0 * bc) / 12.0 + a.sf[i]);
}

// f~_j = W f^E(u_j) + nu A_h u_j at every node; SF_m = sum_j dt s_{m,j} f~_j
// and Y_m = sum_j dt q_{m,j} f~_j (the residual's right-hand side before W^{-1}).
template <int M>
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
        nb9(u, n, x, y, edges, corners);
        double fe_edges = 0.0;
        if (a.fe == ISDC_FE_CUBIC)
            fe_edges = fe_of(at(u, n, x - 1, y), a.fe) + fe_of(at(u, n, x + 1, y), a.fe) +
                       fe_of(at(u, n, x, y - 1), a.fe) + fe_of(at(u, n, x, y + 1), a.fe);
        const double fec = fe_of(uc, a.fe);
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
// (b, k) covers a stride of node a.node[k]'s points.
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

// ---------------------------------------------------------------- compact tail
// One V-cycle of B on levels n_t (<= 63), ..., 1 in one workgroup, every
// level in LDS (same layout and phases as the second-order tail), weighted
// Jacobi smoothing.

template <typename T>
__device__ __forceinline__ T capply_lds(const T* e, int n, int x, int y, int i, T b0, T bf, T bc) {
    T edges = T(0), corners = T(0);
    if (x > 0) edges += e[i - 1];
    if (x < n - 1) edges += e[i + 1];
    if (y > 0) edges += e[i - n];
    if (y < n - 1) edges += e[i + n];
    if (y > 0) {
        if (x > 0) corners += e[i - n - 1];
        if (x < n - 1) corners += e[i - n + 1];
    }
    if (y < n - 1) {
        if (x > 0) corners += e[i + n - 1];
        if (x < n - 1) corners += e[i + n + 1];
    }
    return b0 * e[i] + bf * edges + bc * corners;
}

template <typename T>
__global__ void __launch_bounds__(kTail)
k_ctail(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t, CTailCoefs tc, int nu1, int nu2, double omega,
        int zero_guess) {
    using L = TailLayout<2>;
    __shared__ T le[L::total];
    __shared__ T lr[L::total];
    __shared__ T lt[L::big];
    auto nn = [&](int l) { return ((n_t + 1) >> l) - 1; };
    auto off = [&](int l) {
        int o = 0;
        for (int j = 0; j < l; ++j) o += nn(j) * nn(j);
        return o;
    };
    int nlev = 1;
    while (nn(nlev - 1) > 1) ++nlev;
    {
        constexpr int I = (L::big + kTail - 1) / kTail;
        const int N0 = n_t * n_t;
        T vr[I], ve[I];
#pragma unroll
        for (int it = 0; it < I; ++it) {
            const int i = threadIdx.x + it * kTail;
            vr[it] = i < N0 ? rhs_g[i] : T(0);
            ve[it] = (i < N0 && !zero_guess) ? e_g[i] : T(0);
        }
#pragma unroll
        for (int it = 0; it < I; ++it) {
            const int i = threadIdx.x + it * kTail;
            if (i < N0) {
                lr[i] = vr[it];
                le[i] = ve[it];
            }
        }
    }
    __syncthreads();
    const T w = T(omega);
    const T wts[3] = {T(0.25), T(0.5), T(0.25)};
    auto jacobi = [&](T* e, const T* r, int n, T b0, T bf, T bc) {
        const T inv = T(1) / b0;
        phase<T, 2>(n, lt, [&](bool ok, int x, int y, int, int i, T& v) {
            if (!ok) return false;
            v = e[i] + w * (r[i] - capply_lds(e, n, x, y, i, b0, bf, bc)) * inv;
            return true;
        });
        __syncthreads();
        phase<T, 2>(n, e, [&](bool ok, int, int, int, int i, T& v) {
            if (!ok) return false;
            v = lt[i];
            return true;
        });
        __syncthreads();
    };
    for (int l = 0; l < nlev; ++l) {
        const int n = nn(l);
        const T b0 = T(tc.b0[l]), bf = T(tc.bf[l]), bc = T(tc.bc[l]);
        T* e = le + off(l);
        T* r = lr + off(l);
        if (n == 1) {
            if (threadIdx.x == 0) e[0] = r[0] / b0;
            __syncthreads();
            break;
        }
        for (int k = 0; k < nu1; ++k) jacobi(e, r, n, b0, bf, bc);
        phase<T, 2>(n, lt, [&](bool ok, int x, int y, int, int i, T& v) {
            if (!ok) return false;
            v = r[i] - capply_lds(e, n, x, y, i, b0, bf, bc);
            return true;
        });
        __syncthreads();
        const int nc = (n - 1) / 2;
        T* rc = lr + off(l + 1);
        T* ec = le + off(l + 1);
        phase<T, 2>(nc, rc, [&](bool ok, int X, int Y, int, int I, T& v) {
            if (!ok) return false;
            T acc = T(0);
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const int base = (2 * Y + oy) * n + 2 * X;
                acc += wts[oy] * (wts[0] * lt[base] + wts[1] * lt[base + 1] + wts[2] * lt[base + 2]);
            }
            v = acc;
            ec[I] = T(0);
            return true;
        });
        __syncthreads();
    }
    for (int l = nlev - 2; l >= 0; --l) {
        const int n = nn(l);
        const int nc = nn(l + 1);
        const T b0 = T(tc.b0[l]), bf = T(tc.bf[l]), bc = T(tc.bc[l]);
        T* e = le + off(l);
        T* r = lr + off(l);
        const T* ec = le + off(l + 1);
        phase<T, 2>(n, e, [&](bool ok, int x, int y, int, int i, T& v) {
            if (!ok) return false;
            v = e[i] + interp_at<T, 2>(ec, nc, x, y, 0);
            return true;
        });
        __syncthreads();
        for (int k = 0; k < nu2; ++k) jacobi(e, r, n, b0, bf, bc);
    }
    {
        constexpr int I = (L::big + kTail - 1) / kTail;
        const int N0 = n_t * n_t;
#pragma unroll
        for (int it = 0; it < I; ++it) {
            const int i = threadIdx.x + it * kTail;
            if (i < N0) e_g[i] = le[i];
        }
    }
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
hipError_t launch_cjacobi(int n, const CCoef<T>& k, bool zero, const T* r, const T* e_in, T* e_out, hipStream_t s) {
    if (zero)
        hipLaunchKernelGGL((k_cjacobi<T, true>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
    else
        hipLaunchKernelGGL((k_cjacobi<T, false>), grid2(n), dim3(kB), 0, s, r, e_in, e_out, n, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cresfw(int n, const CCoef<T>& k, const T* r, const T* e, T* rc, hipStream_t s) {
    hipLaunchKernelGGL((k_cresfw<T>), grid2((n - 1) / 2), dim3(kB), 0, s, r, e, rc, n, k);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cresnorm(int n, const CCoef<T>& k, const T* r, const T* e, double* partial, int* nblocks,
                           hipStream_t s) {
    const dim3 g = grid2(n);
    *nblocks = (int)(g.x * g.y);
    hipLaunchKernelGGL((k_cresnorm<T>), g, dim3(kB), 0, s, r, e, n, k, partial);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_crhs(const CRhsArgs& a, T* out, hipStream_t s) {
    hipLaunchKernelGGL((k_crhs<T>), grid2(a.n), dim3(kB), 0, s, a, out);
    return hipGetLastError();
}

hipError_t launch_cquad(const CQuadArgs& a, int M, hipStream_t s) {
    switch (M) {
#define ISDC_CQ(MM) case MM: hipLaunchKernelGGL((k_cquad<MM>), grid2(a.n), dim3(kB), 0, s, a); break;
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

template <typename T>
hipError_t launch_ctail(const MGConfig& mg, int n, double c, double w, double h, bool zero, const T* rhs, T* e,
                        hipStream_t s) {
    if (n > TailLayout<2>::nmax) return hipErrorInvalidValue;
    CTailCoefs tc;
    double H = h;
    for (int l = 0; l < 16; ++l) {
        const CCoef<double> k = make_ccoef<double>(c, w, H, 1.0);
        tc.b0[l] = k.b0;
        tc.bf[l] = k.bf;
        tc.bc[l] = k.bc;
        H *= 2.0;
    }
    hipLaunchKernelGGL((k_ctail<T>), dim3(1), dim3(kTail), 0, s, rhs, e, n, tc, mg.nu_pre, mg.nu_post, mg.omega,
                       zero ? 1 : 0);
    return hipGetLastError();
}

#define ISDC_CINST(T)                                                                                          \
    template CCoef<T> make_ccoef<T>(double, double, double, double);                                           \
    template hipError_t launch_cjacobi<T>(int, const CCoef<T>&, bool, const T*, const T*, T*, hipStream_t);     \
    template hipError_t launch_cresfw<T>(int, const CCoef<T>&, const T*, const T*, T*, hipStream_t);            \
    template hipError_t launch_cresnorm<T>(int, const CCoef<T>&, const T*, const T*, double*, int*, hipStream_t); \
    template hipError_t launch_crhs<T>(const CRhsArgs&, T*, hipStream_t);                                      \
    template hipError_t launch_ctail<T>(const MGConfig&, int, double, double, double, bool, const T*, T*, hipStream_t);
ISDC_CINST(float)
ISDC_CINST(double)
#undef ISDC_CINST

}  // namespace isdc
