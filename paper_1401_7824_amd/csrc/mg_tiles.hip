// LDS-tiled multigrid kernels for A_l = I - c L_{h_l} (Sec. 3: the implicit
// systems of eq. (4) are solved with multigrid V-cycles) and the coarse tail.
//
// Every multi-workgroup kernel works on one tile of the grid per workgroup:
// it stages the tile plus a halo in LDS, does all its arithmetic there and
// writes only its own tile, so each array element comes from HBM about once.
//
//   k_rbgs_tile         one complete red-black Gauss-Seidel step (red on the
//                       tile plus a halo of 1, black on the tile), out of place;
//   k_restrict_tile     residual rhs - A e and its full-weighting restriction;
//   k_prolong_rbgs_tile e + P e_c (linear interpolation) followed by one
//                       red-black step; optionally writes g + e to a float64
//                       node array instead of e (the node update of eq. (4));
//   k_march_rbgs        the 3D form of the two red-black kernels above:
//                       columns of planes marched in z instead of 3D tiles;
//   k_march_restrict    the 3D restriction of those levels, marched over
//                       coarse planes;
//   k_rows_*            the 2D forms of the red-black, fused red-black +
//                       restriction and prolongation + red-black kernels on
//                       row-mapped tiles (rows2d.h), and the first launch of
//                       a solve with the right-hand side of eq. (4) formed in
//                       it (k_rows_rhs_rbgs_restrict).
//
// Workgroups are numbered so that each of the 8 XCDs (the hardware hands
// workgroup b to XCD b mod 8) receives a contiguous band of tiles, keeping the
// halo re-reads inside one XCD's L2.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "mg_device.h"
#include "mg_march.h"
#include "rows2d.h"
#include "sdc_device.h"
#include "tailc.h"

namespace isdc {

namespace {

template <typename T, int D, bool ZERO, int S>
__global__ void __launch_bounds__(kThreads)
k_rbgs_tile(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, int ntx, int nty,
            T a, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using TL = TileS<D, S>;
    int x0, y0, z0;
    tile_origin(ntx, nty, TL::X, TL::Y, TL::Z, x0, y0, z0);
    rbgs_tile_body<T, D, ZERO, TL>(r, e_in, e_out, n, x0, y0, z0, a, invdiag);
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads)
k_restrict_tile(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc, int n, int ntx, int nty,
                T a, T diag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int X0, Y0, Z0;
    tile_origin(ntx, nty, CTile<D>::X, CTile<D>::Y, CTile<D>::Z, X0, Y0, Z0);
    restrict_tile_body<T, D>(r, e, rc, n, X0, Y0, Z0, a, diag);
}

template <typename T, int D, bool ZERO, int S>
__global__ void __launch_bounds__(kThreads)
k_rbgs_restrict_tile(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, T* __restrict__ rc,
                     int n, int ntx, int nty, T a, T diag, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using TL = TileS<D, S>;
    int x0, y0, z0;
    tile_origin(ntx, nty, TL::X, TL::Y, TL::Z, x0, y0, z0);
    rbgs_restrict_body<T, D, ZERO, TL>(r, e_in, e_out, rc, n, x0, y0, z0, a, diag, invdiag);
}

template <typename T, int D, int MODE, int S>
__global__ void __launch_bounds__(kThreads)
k_prolong_rbgs_tile(const T* __restrict__ r, const T* __restrict__ e_in, const T* __restrict__ ec, T* __restrict__ e_out,
                    int n, int ntx, int nty, T a, T invdiag, const double* __restrict__ g, double* __restrict__ u_out, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using TL = TileS<D, S>;
    int x0, y0, z0;
    tile_origin(ntx, nty, TL::X, TL::Y, TL::Z, x0, y0, z0);
    prolong_rbgs_body<T, D, MODE, TL>(r, e_in, ec, e_out, n, x0, y0, z0, a, invdiag, g, u_out);
}

// 3D red-black step (optionally after the prolongation, with the node
// update) by z-marching columns of mz planes (march_depth of the level).
template <typename T, bool PRO, int MODE, bool ZERO>
__global__ void __launch_bounds__(kThreads)
k_march_rbgs(const T* __restrict__ r, const T* __restrict__ e_in, const T* __restrict__ ec, T* __restrict__ e_out,
             int n, int ntx, int nty, int mz, T a, T invdiag, const double* __restrict__ g, double* __restrict__ u_out, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int x0, y0, z0;
    tile_origin(ntx, nty, MTile<T>::X, MTile<T>::Y, mz, x0, y0, z0);
    march_rbgs_body<T, PRO, MODE, ZERO>(r, e_in, ec, e_out, n, x0, y0, z0, mz, a, invdiag, g, u_out);
}

// 2D row-mapped tiles (shape S selects the row tile).
// 3D residual + full weighting, z-marched over coarse planes (levels of
// 127^3 and up).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_march_restrict(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc, int n, int ntx, int nty,
                 int mzc, T a, T diag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int X0, Y0, Z0;
    tile_origin(ntx, nty, MRTile::X, MRTile::Y, mzc, X0, Y0, Z0);
    march_restrict_body<T>(r, e, rc, n, X0, Y0, Z0, mzc, a, diag);
}

// 3D zero-start red-black step fused with the residual and full weighting,
// z-marched over coarse planes (levels of 127^3 and up): writes the iterate
// and the coarse rhs.
template <typename T>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_march_zrestrict(const T* __restrict__ r, T* __restrict__ e_out, T* __restrict__ rc, int n, int ntx, int nty, int mzc,
                  T a, T diag, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int X0, Y0, Z0;
    tile_origin(ntx, nty, MRTile::X, MRTile::Y, mzc, X0, Y0, Z0);
    march_zrestrict_body<T>(r, e_out, rc, n, X0, Y0, Z0, mzc, a, diag, invdiag);
}

// 3D red-black step from a nonzero iterate fused with the residual and full
// weighting, z-marched over coarse planes (levels of 127^3 and up): writes
// the iterate and the coarse rhs.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_march_srestrict(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, T* __restrict__ rc, int n,
                  int ntx, int nty, int mzc, T a, T diag, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int X0, Y0, Z0;
    tile_origin(ntx, nty, MRTile::X, MRTile::Y, mzc, X0, Y0, Z0);
    march_srestrict_body<T>(r, e_in, e_out, rc, n, X0, Y0, Z0, mzc, a, diag, invdiag);
}

template <typename T, bool ZERO, int S>
__global__ void __launch_bounds__(kThreads)
k_rows_rbgs(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, int ntx, int nty, T a,
            T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using RT = typename RowShape<S>::RT;
    int x0, y0, z0;
    tile_origin(ntx, nty, RT::TX, RT::TY, 1, x0, y0, z0);
    rows_rbgs_body<T, ZERO, RT>(r, e_in, e_out, n, x0, y0, a, invdiag);
}

template <typename T, bool ZERO, int S>
__global__ void __launch_bounds__(kThreads)
k_rows_rbgs_restrict(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, T* __restrict__ rc,
                     int n, int ntx, int nty, T a, T diag, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using RT = typename RowShape<S>::RT;
    int x0, y0, z0;
    tile_origin(ntx, nty, RT::TX, RT::TY, 1, x0, y0, z0);
    rows_rbgs_restrict_body<T, ZERO, RT>(r, e_in, e_out, rc, n, x0, y0, a, diag, invdiag);
}

template <typename T, int S>
__global__ void __launch_bounds__(kThreads)
k_rows_rhs_rbgs_restrict(RhsArgs ra, T* __restrict__ r, T* __restrict__ e_out, T* __restrict__ rc, int n, int ntx,
                         int nty, T a, T diag, T invdiag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using RT = typename RowShape<S>::RT;
    int x0, y0, z0;
    tile_origin(ntx, nty, RT::TX, RT::TY, 1, x0, y0, z0);
    const int fe = ra.fe;
    rows_rhs_rbgs_restrict_body<T, RT>(ra.um_new, ra.um_old, ra.up_old, ra.sf, ra.dtm, fe != ISDC_FE_ZERO,
                                       [fe](double u) { return fexp(u, fe); }, r, e_out, rc, n, x0, y0, a, diag,
                                       invdiag);
}

template <typename T, int MODE, int S>
__global__ void __launch_bounds__(kThreads)
k_rows_prolong_rbgs(const T* __restrict__ r, const T* __restrict__ e_in, const T* __restrict__ ec,
                    T* __restrict__ e_out, int n, int ntx, int nty, T a, T invdiag, const double* __restrict__ g,
                    double* __restrict__ u_out, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    using RT = typename RowShape<S>::RT;
    int x0, y0, z0;
    tile_origin(ntx, nty, RT::TX, RT::TY, 1, x0, y0, z0);
    rows_prolong_rbgs_body<T, MODE, RT>(r, e_in, ec, e_out, n, x0, y0, a, invdiag, g, u_out);
}

template <typename T, int D>
__global__ void __launch_bounds__(kTail)
k_tail(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t, TailCoefs tc, int smoother, int nu1, int nu2,
       double omega, int zero_guess, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    tailc_body<T, D>(rhs_g, e_g, n_t, tc, smoother, nu1, nu2, omega, zero_guess);
}

}  // namespace

#define ISDC_DISPATCH_D(d, ...)                              \
    switch (d) {                                             \
        case 1: { constexpr int D = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int D = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int D = 3; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                \
    }

// dimension (1 or 3; 2D levels run the row kernels) and tile shape
// (0 .. kShapes-1) as compile-time constants D, S
#define ISDC_DISPATCH_DS(d, shape, ...)                                            \
    switch ((d) * 4 + (shape)) {                                                   \
        case 4: { constexpr int D = 1, S = 0; __VA_ARGS__; } break;                \
        case 5: { constexpr int D = 1, S = 1; __VA_ARGS__; } break;                \
        case 6: { constexpr int D = 1, S = 2; __VA_ARGS__; } break;                \
        case 12: { constexpr int D = 3, S = 0; __VA_ARGS__; } break;               \
        case 13: { constexpr int D = 3, S = 1; __VA_ARGS__; } break;               \
        case 14: { constexpr int D = 3, S = 2; __VA_ARGS__; } break;               \
        default: return hipErrorInvalidValue;                                      \
    }

// 2D row shape as the compile-time constant S
#define ISDC_DISPATCH_ROWS(shape, ...)                                  \
    switch (shape) {                                                    \
        case 0: { constexpr int S = 0; __VA_ARGS__; } break;            \
        case 1: { constexpr int S = 1; __VA_ARGS__; } break;            \
        case 2: { constexpr int S = 2; __VA_ARGS__; } break;            \
        default: return hipErrorInvalidValue;                           \
    }

// Workgroups of one z-march kernel that are resident on the device at once
// (its occupancy per CU from the compiled kernel's registers and LDS, times
// the CUs), read once per kernel; 0 if the runtime cannot say.
template <typename T, bool PRO, int MODE, bool ZERO>
int march_resident() {
    static const int v = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_march_rbgs<T, PRO, MODE, ZERO>, kThreads, 0) !=
            hipSuccess)
            return 0;
        return per * cus;
    }();
    return v;
}

// Column depth of a marched level for tile shape `shape`: shapes 0 and 2 as
// march_depth (16 / 8 planes at 255^3); shape 1 the even depth at which all
// columns of the level fit in one round of resident workgroups, so that no
// second, partly empty round follows the first.
inline int march_depth_fitted(int n, int shape, int nxy, int resident) {
    if (shape != 1 || resident <= 0) return march_depth(n, shape);
    const int cols = std::max(1, resident / nxy);
    int dz = (n + cols - 1) / cols;
    dz += dz & 1;
    return std::max(2, dz);
}

template <typename T, bool PRO, int MODE, bool ZERO>
int march_depth_of(int n, int shape) {
    int ntx, nty, nb;
    tile_counts<3>(n, MTile<T>::X, MTile<T>::Y, n, ntx, nty, nb);
    return march_depth_fitted(n, shape, ntx * nty, shape == 1 ? march_resident<T, PRO, MODE, ZERO>() : 0);
}

// Coarse planes per column of the fused red-black step + restriction (ZERO:
// from a zero iterate): the depth at which all columns fit in one round of
// resident workgroups, at least 4.
template <typename T, bool ZERO>
int frestrict_depth(int nc, int nxy) {
    static const int resident = [] {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
        hipError_t e;
        if constexpr (ZERO)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_march_zrestrict<T>, kThreads, 0);
        else
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_march_srestrict<T>, kThreads, 0);
        if (e != hipSuccess) return 0;
        return per * cus;
    }();
    if (resident <= 0) return march_restrict_depth();
    const int cols = std::max(1, resident / nxy);
    return std::max(4, (nc + cols - 1) / cols);
}

template <typename T>
hipError_t launch_rbgs_tile(int d, int n, const Coef<T>& co, bool zero, const T* r, const T* e_in, T* e_out,
                            hipStream_t s, int shape) {
    if (d == 3 && march_depth(n) > 0) {
        if (shape < 0 || shape >= kShapes) return hipErrorInvalidValue;
        const int mz = zero ? march_depth_of<T, false, 0, true>(n, shape) : march_depth_of<T, false, 0, false>(n, shape);
        int ntx, nty, nb;
        tile_counts<3>(n, MTile<T>::X, MTile<T>::Y, mz, ntx, nty, nb);
        if (zero)
            ISDC_GLAUNCH((k_march_rbgs<T, false, 0, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, (const T*)nullptr, e_out, n, ntx, nty, mz, co.a, co.invdiag, (const double*)nullptr, (double*)nullptr);
        else
            ISDC_GLAUNCH((k_march_rbgs<T, false, 0, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, (const T*)nullptr, e_out, n, ntx, nty, mz, co.a, co.invdiag, (const double*)nullptr, (double*)nullptr);
        return hipGetLastError();
    }
    if (d == 2) {
        ISDC_DISPATCH_ROWS(shape, {
            using RT = typename RowShape<S>::RT;
            int ntx, nty, nb;
            tile_counts<2>(n, RT::TX, RT::TY, 1, ntx, nty, nb);
            if (zero)
                ISDC_GLAUNCH((k_rows_rbgs<T, true, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
            else
                ISDC_GLAUNCH((k_rows_rbgs<T, false, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
        });
        return hipGetLastError();
    }
    ISDC_DISPATCH_DS(d, shape, {
        using TL = TileS<D, S>;
        int ntx, nty, nb;
        tile_counts<D>(n, TL::X, TL::Y, TL::Z, ntx, nty, nb);
        if (zero)
            ISDC_GLAUNCH((k_rbgs_tile<T, D, true, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
        else
            ISDC_GLAUNCH((k_rbgs_tile<T, D, false, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_tile(int d, int n, const Coef<T>& co, const T* r, const T* e, T* rc, hipStream_t s) {
    const int nc = (n - 1) / 2;
    if (d == 3 && march_depth(n) > 0) {
        const int mzc = march_restrict_depth();
        int ntx, nty, nb;
        tile_counts<3>(nc, MRTile::X, MRTile::Y, mzc, ntx, nty, nb);
        ISDC_GLAUNCH((k_march_restrict<T>), dim3(nb), dim3(kThreads), 0, s, r, e, rc, n, ntx, nty, mzc, co.a,
                           co.diag);
        return hipGetLastError();
    }
    ISDC_DISPATCH_D(d, {
        int ntx, nty, nb;
        tile_counts<D>(nc, CTile<D>::X, CTile<D>::Y, CTile<D>::Z, ntx, nty, nb);
        ISDC_GLAUNCH((k_restrict_tile<T, D>), dim3(nb), dim3(kThreads), 0, s, r, e, rc, n, ntx, nty, co.a, co.diag);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rbgs_restrict_tile(int d, int n, const Coef<T>& co, bool zero, const T* r, const T* e_in, T* e_out,
                                     T* rc, hipStream_t s, int shape) {
    if (d == 3) {
        // 3D: z-marched levels only (the 3D tiles would need a halo of 3)
        if (march_depth(n) <= 0) return hipErrorInvalidValue;
        const int nc = (n - 1) / 2;
        int ntx, nty, nb;
        tile_counts<3>(nc, MRTile::X, MRTile::Y, nc, ntx, nty, nb);
        const int mzc = zero ? frestrict_depth<T, true>(nc, ntx * nty) : frestrict_depth<T, false>(nc, ntx * nty);
        tile_counts<3>(nc, MRTile::X, MRTile::Y, mzc, ntx, nty, nb);
        if (zero)
            ISDC_GLAUNCH((k_march_zrestrict<T>), dim3(nb), dim3(kThreads), 0, s, r, e_out, rc, n, ntx, nty, mzc, co.a,
                         co.diag, co.invdiag);
        else
            ISDC_GLAUNCH((k_march_srestrict<T>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, mzc,
                         co.a, co.diag, co.invdiag);
        return hipGetLastError();
    }
    if (d == 2) {
        ISDC_DISPATCH_ROWS(shape, {
            using RT = typename RowShape<S>::RT;
            int ntx, nty, nb;
            tile_counts<2>(n, RT::TX, RT::TY, 1, ntx, nty, nb);
            if (zero)
                ISDC_GLAUNCH((k_rows_rbgs_restrict<T, true, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, co.a, co.diag, co.invdiag);
            else
                ISDC_GLAUNCH((k_rows_rbgs_restrict<T, false, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, co.a, co.diag, co.invdiag);
        });
        return hipGetLastError();
    }
    ISDC_DISPATCH_DS(d, shape, {
        if constexpr (D < 3) {
            using TL = TileS<D, S>;
            int ntx, nty, nb;
            tile_counts<D>(n, TL::X, TL::Y, TL::Z, ntx, nty, nb);
            if (zero)
                ISDC_GLAUNCH((k_rbgs_restrict_tile<T, D, true, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, co.a, co.diag, co.invdiag);
            else
                ISDC_GLAUNCH((k_rbgs_restrict_tile<T, D, false, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, rc, n, ntx, nty, co.a, co.diag, co.invdiag);
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rhs_rbgs_restrict_tile(int d, int n, const RhsArgs& ra, const Coef<T>& co, T* r, T* e_out, T* rc,
                                         hipStream_t s, int shape) {
    if (d != 2 || ra.guess != ISDC_GUESS_PREV_SWEEP || ra.n != n) return hipErrorInvalidValue;
    ISDC_DISPATCH_ROWS(shape, {
        using RT = typename RowShape<S>::RT;
        int ntx, nty, nb;
        tile_counts<2>(n, RT::TX, RT::TY, 1, ntx, nty, nb);
        ISDC_GLAUNCH((k_rows_rhs_rbgs_restrict<T, S>), dim3(nb), dim3(kThreads), 0, s, ra, r, e_out, rc, n, ntx, nty, co.a, co.diag, co.invdiag);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_rbgs_tile(int d, int n, const Coef<T>& co, const T* r, const T* e_in, const T* ec,
                                    T* e_out, const double* g, double* u_out, int mode, hipStream_t s, int shape) {
    if (d == 3 && march_depth(n) > 0) {
        if (shape < 0 || shape >= kShapes) return hipErrorInvalidValue;
        const int mz = mode == 0 ? march_depth_of<T, true, 0, false>(n, shape)
                                 : (mode == 1 ? march_depth_of<T, true, 1, false>(n, shape)
                                              : march_depth_of<T, true, 2, false>(n, shape));
        int ntx, nty, nb;
        tile_counts<3>(n, MTile<T>::X, MTile<T>::Y, mz, ntx, nty, nb);
        if (mode == 0)
            ISDC_GLAUNCH((k_march_rbgs<T, true, 0, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, mz, co.a, co.invdiag, g, u_out);
        else if (mode == 1)
            ISDC_GLAUNCH((k_march_rbgs<T, true, 1, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, mz, co.a, co.invdiag, g, u_out);
        else
            ISDC_GLAUNCH((k_march_rbgs<T, true, 2, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, mz, co.a, co.invdiag, g, u_out);
        return hipGetLastError();
    }
    if (d == 2) {
        ISDC_DISPATCH_ROWS(shape, {
            using RT = typename RowShape<S>::RT;
            int ntx, nty, nb;
            tile_counts<2>(n, RT::TX, RT::TY, 1, ntx, nty, nb);
            if (mode == 0)
                ISDC_GLAUNCH((k_rows_prolong_rbgs<T, 0, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
            else if (mode == 1)
                ISDC_GLAUNCH((k_rows_prolong_rbgs<T, 1, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
            else
                ISDC_GLAUNCH((k_rows_prolong_rbgs<T, 2, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
        });
        return hipGetLastError();
    }
    ISDC_DISPATCH_DS(d, shape, {
        using TL = TileS<D, S>;
        int ntx, nty, nb;
        tile_counts<D>(n, TL::X, TL::Y, TL::Z, ntx, nty, nb);
        if (mode == 0)
            ISDC_GLAUNCH((k_prolong_rbgs_tile<T, D, 0, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
        else if (mode == 1)
            ISDC_GLAUNCH((k_prolong_rbgs_tile<T, D, 1, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
        else
            ISDC_GLAUNCH((k_prolong_rbgs_tile<T, D, 2, S>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
    });
    return hipGetLastError();
}

static_assert(kShapes == kTileShapes, "tile shape count of the kernels and of the launchers");

int tail_max_n(int d) {
    return d == 1 ? kTailMax<1> : (d == 2 ? kTailMax<2> : kTailMax<3>);
}

template <typename T>
hipError_t launch_tail(const MGConfig& cfg, int n, double c, double h, bool zero_guess, const T* rhs, T* e,
                       hipStream_t s) {
    if (n < 1 || n > tail_max_n(cfg.d) || ((n + 1) & n) != 0) return hipErrorInvalidValue;  // n = 2^k - 1
    TailCoefs tc;
    double hl = h;
    for (int l = 0, m = n; l < 16; ++l, m = (m - 1) / 2, hl *= 2.0) {
        const Coef<double> co = make_coef<double>(c, hl, cfg.d, cfg.omega);
        tc.a[l] = co.a;
        tc.diag[l] = co.diag;
        tc.invdiag[l] = co.invdiag;
        if (m == 1) break;
    }
    ISDC_DISPATCH_D(cfg.d, {
        ISDC_GLAUNCH((k_tail<T, D>), dim3(1), dim3(kTail), 0, s, rhs, e, n, tc, cfg.smoother, cfg.nu_pre,
                           cfg.nu_post, cfg.omega, zero_guess ? 1 : 0);
    });
    return hipGetLastError();
}

bool rbgs_restrict_fused(int d, int n) { return d <= 2 || (d == 3 && march_depth(n) > 0); }

#define ISDC_INST_T(T)                                                                                          \
    template hipError_t launch_rbgs_tile<T>(int, int, const Coef<T>&, bool, const T*, const T*, T*, hipStream_t, int); \
    template hipError_t launch_restrict_tile<T>(int, int, const Coef<T>&, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_rbgs_restrict_tile<T>(int, int, const Coef<T>&, bool, const T*, const T*, T*, T*,    \
                                                     hipStream_t, int);                                            \
    template hipError_t launch_prolong_rbgs_tile<T>(int, int, const Coef<T>&, const T*, const T*, const T*, T*,  \
                                                    const double*, double*, int, hipStream_t, int);             \
    template hipError_t launch_rhs_rbgs_restrict_tile<T>(int, int, const RhsArgs&, const Coef<T>&, T*, T*, T*,   \
                                                         hipStream_t, int);                                     \
    template hipError_t launch_tail<T>(const MGConfig&, int, double, double, bool, const T*, T*, hipStream_t);

ISDC_INST_T(float)
ISDC_INST_T(double)

}  // namespace isdc
