// Geometric multigrid kernels for A_l = I - c L_{h_l} (Sec. 3: the implicit
// Euler systems of eq. (4) are solved with spatial multigrid; ISDC uses a
// fixed small number of V-cycles).
//
// Layout: dense n^d arrays of interior points, x fastest; ghosts are implicit
// zeros (homogeneous Dirichlet).  Grid of a stencil launch: blockDim = 256
// along x, gridDim = (ceil(points-per-row / 256), rows, planes).
//
// Components (the paper leaves them open; these are the textbook choices):
//   smoothers  -- red-black Gauss-Seidel (red = even index sum, updated first)
//                 or weighted Jacobi;
//   restriction -- full weighting (1/4, 1/2, 1/4 per axis) of the residual;
//   prolongation -- (bi/tri)linear interpolation added to the iterate;
// These are the plain one-thread-per-point forms, used for the Jacobi
// smoother, in-place red-black half steps and the residual norm; the tiled
// kernels and the coarse tail live in mg_tiles.hip.
#include <hip/hip_runtime.h>
#include <cmath>

#include "internal.h"

namespace isdc {

namespace {

constexpr int kBlock = 256;

template <int D>
__device__ __forceinline__ void coords(int n, int& x, int& y, int& z, int per_row_thread) {
    x = per_row_thread;
    y = (D >= 2) ? (int)blockIdx.y : 0;
    z = (D == 3) ? (int)blockIdx.z : 0;
}

template <int D>
__device__ __forceinline__ size_t lin(int n, int x, int y, int z) {
    if (D == 1) return (size_t)x;
    if (D == 2) return (size_t)y * n + x;
    return ((size_t)z * n + y) * n + x;
}

// Sum of the 2d neighbours of point (x,y,z) with zero ghosts.
template <typename T, int D>
__device__ __forceinline__ T nbsum(const T* __restrict__ u, int n, int x, int y, int z, size_t i) {
    T s = T(0);
    if (x > 0) s += u[i - 1];
    if (x < n - 1) s += u[i + 1];
    if (D >= 2) {
        if (y > 0) s += u[i - n];
        if (y < n - 1) s += u[i + n];
    }
    if (D == 3) {
        size_t nn = (size_t)n * n;
        if (z > 0) s += u[i - nn];
        if (z < n - 1) s += u[i + nn];
    }
    return s;
}

// ---------------------------------------------------------------- smoothers

template <typename T, int D, bool ZERO>
__global__ void __launch_bounds__(kBlock)
k_jacobi(const T* __restrict__ rhs, const T* __restrict__ u, T* __restrict__ out, int n, T a, T diag,
         T invdiag, T w, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int x, y, z;
    coords<D>(n, x, y, z, blockIdx.x * kBlock + threadIdx.x);
    if (x >= n) return;
    size_t i = lin<D>(n, x, y, z);
    T r = rhs[i];
    if (ZERO) {
        out[i] = w * (r * invdiag);
        return;
    }
    T c = u[i];
    T Au = diag * c - a * nbsum<T, D>(u, n, x, y, z, i);
    out[i] = c + w * ((r - Au) * invdiag);
}

// Half of a red-black Gauss-Seidel step, in place: the points of `colour`
// ((x+y+z) % 2 == colour) are set to (rhs + a * neighbour sum) / diag.
// Thread j of a row owns x = 2j and 2j+1.  ZERO (red pass on a zero iterate):
// red points get rhs / diag and black points are cleared.
template <typename T, int D, bool ZERO>
__global__ void __launch_bounds__(kBlock)
k_rbgs_half(const T* __restrict__ rhs, T* __restrict__ u, int n, T a, T invdiag, int colour, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    int j, y, z;
    coords<D>(n, j, y, z, blockIdx.x * kBlock + threadIdx.x);
    int par = (colour + y + z) & 1;
    int x = 2 * j + par;
    if (ZERO) {
        int xo = 2 * j + (par ^ 1);
        if (xo < n) u[lin<D>(n, xo, y, z)] = T(0);
        if (x < n) {
            size_t i = lin<D>(n, x, y, z);
            u[i] = rhs[i] * invdiag;
        }
        return;
    }
    if (x >= n) return;
    size_t i = lin<D>(n, x, y, z);
    u[i] = (rhs[i] + a * nbsum<T, D>(u, n, x, y, z, i)) * invdiag;
}

// ---------------------------------------------------------------- transfers

template <typename T, int D>
__device__ __forceinline__ T residual_at(const T* __restrict__ rhs, const T* __restrict__ u, int n,
                                         int x, int y, int z, T a, T diag) {
    size_t i = lin<D>(n, x, y, z);
    return rhs[i] - (diag * u[i] - a * nbsum<T, D>(u, n, x, y, z, i));
}

// One thread per coarse point (X,Y,Z); the fine centre is (2X+1, 2Y+1, 2Z+1).
template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_restrict(const T* __restrict__ rhs, const T* __restrict__ u, T* __restrict__ rc, int n, T a, T diag, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    const int nc = (n - 1) / 2;
    int X, Y, Z;
    coords<D>(nc, X, Y, Z, blockIdx.x * kBlock + threadIdx.x);
    if (X >= nc) return;
    const T wt[3] = {T(0.25), T(0.5), T(0.25)};
    T acc = T(0);
    const int zlo = (D == 3) ? -1 : 0, zhi = (D == 3) ? 1 : 0;
    const int ylo = (D >= 2) ? -1 : 0, yhi = (D >= 2) ? 1 : 0;
    for (int oz = zlo; oz <= zhi; ++oz) {
        for (int oy = ylo; oy <= yhi; ++oy) {
            T row = T(0);
            for (int ox = -1; ox <= 1; ++ox) {
                int x = 2 * X + 1 + ox;
                int y = (D >= 2) ? 2 * Y + 1 + oy : 0;
                int z = (D == 3) ? 2 * Z + 1 + oz : 0;
                row += wt[ox + 1] * residual_at<T, D>(rhs, u, n, x, y, z, a, diag);
            }
            T wyz = (D >= 2 ? wt[oy + 1] : T(1)) * (D == 3 ? wt[oz + 1] : T(1));
            acc += wyz * row;
        }
    }
    rc[lin<D>(nc, X, Y, Z)] = acc;
}

// Interpolation weights along one axis for fine index i: odd i -> coarse
// (i-1)/2 with weight 1; even i -> coarse i/2-1 and i/2 with weight 1/2 each
// (indices outside [0, nc) are boundary zeros).
__device__ __forceinline__ int interp_taps(int i, int nc, int* idx, float* w) {
    if (i & 1) {
        idx[0] = (i - 1) >> 1;
        w[0] = 1.0f;
        return 1;
    }
    int k = 0;
    int lo = (i >> 1) - 1, hi = i >> 1;
    if (lo >= 0) { idx[k] = lo; w[k] = 0.5f; ++k; }
    if (hi < nc) { idx[k] = hi; w[k] = 0.5f; ++k; }
    return k;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_prolong(const T* __restrict__ ec, T* __restrict__ u, int n, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    const int nc = (n - 1) / 2;
    int x, y, z;
    coords<D>(n, x, y, z, blockIdx.x * kBlock + threadIdx.x);
    if (x >= n) return;
    int ix[2], iy[2] = {0, 0}, iz[2] = {0, 0};
    float wx[2], wy[2] = {1.f, 1.f}, wz[2] = {1.f, 1.f};
    int kx = interp_taps(x, nc, ix, wx);
    int ky = (D >= 2) ? interp_taps(y, nc, iy, wy) : 1;
    int kz = (D == 3) ? interp_taps(z, nc, iz, wz) : 1;
    T acc = T(0);
    for (int c = 0; c < kz; ++c)
        for (int b = 0; b < ky; ++b)
            for (int a = 0; a < kx; ++a)
                acc += T(wx[a]) * T(wy[b]) * T(wz[c]) * ec[lin<D>(nc, ix[a], iy[b], iz[c])];
    u[lin<D>(n, x, y, z)] += acc;
}

// ---------------------------------------------------------------- reductions

__device__ __forceinline__ double nanmax(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

// Block-wide NaN-propagating max; result valid in thread 0.
__device__ double block_max(double v) {
    __shared__ double sh[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i) v = nanmax(v, sh[i]);
    }
    return v;
}

template <typename T, int D>
__global__ void __launch_bounds__(kBlock)
k_resnorm(const T* __restrict__ rhs, const T* __restrict__ u, int n, T a, T diag, double* partial, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    const size_t N = (D == 1) ? (size_t)n : (D == 2 ? (size_t)n * n : (size_t)n * n * n);
    double m = 0.0;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
        int x = (int)(i % n);
        size_t t = i / n;
        int y = (D >= 2) ? (int)(t % n) : 0;
        int z = (D == 3) ? (int)(t / n) : 0;
        T r = residual_at<T, D>(rhs, u, n, x, y, z, a, diag);
        m = nanmax(m, fabs((double)r));
    }
    m = block_max(m);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// Max over nb per-workgroup partial maxima, one thread's share: eight independent loads in flight per
// pass (the partials come from tens of thousands of workgroups, and one load at a time would leave the
// single reducing workgroup waiting on L2 latency once per 256 values).
__device__ __forceinline__ double partials_share_max(const double* __restrict__ partial, int nb) {
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int i = threadIdx.x;
    for (; i + 7 * kBlock < nb; i += 8 * kBlock) {
#pragma unroll
        for (int k = 0; k < 8; ++k) m[k] = nanmax(m[k], partial[i + k * kBlock]);
    }
    for (; i < nb; i += kBlock) m[0] = nanmax(m[0], partial[i]);
#pragma unroll
    for (int k = 1; k < 8; ++k) m[0] = nanmax(m[0], m[k]);
    return m[0];
}

__global__ void __launch_bounds__(kBlock)
k_reduce_max(const double* __restrict__ partial, int nb, double* __restrict__ out) {
    double m = partials_share_max(partial, nb);
    m = block_max(m);
    if (threadIdx.x == 0) out[0] = m;
}

__global__ void __launch_bounds__(64) k_gate_reset(int* __restrict__ gate) {
    if (threadIdx.x < 2) gate[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(kBlock)
k_reduce_gate(const double* __restrict__ partial, int nb, double tol, int limit, int count_cycle, int* __restrict__ gate,
              double* __restrict__ res_out) {
    if (gate[0]) return;
    double m = partials_share_max(partial, nb);
    m = block_max(m);
    if (threadIdx.x == 0) {
        res_out[0] = m;
        if (m <= tol || gate[1] >= limit) gate[0] = 1;
        else if (count_cycle) gate[1] += 1;
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ p, size_t count, T v, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(const T* __restrict__ s, T* __restrict__ d, size_t count, const int* __restrict__ gate) {
    if (gate && *gate) return;  // the solve met its tolerance on the device
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += (size_t)gridDim.x * kBlock)
        d[i] = s[i];
}

inline dim3 stencil_grid(int d, int per_row, int n) {
    return dim3((unsigned)((per_row + kBlock - 1) / kBlock), d >= 2 ? (unsigned)n : 1u, d == 3 ? (unsigned)n : 1u);
}

inline int reduce_blocks(size_t N) {
    size_t b = (N + kBlock - 1) / kBlock;
    return (int)(b < (size_t)kReduceBlocks ? b : (size_t)kReduceBlocks);
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T>
Coef<T> make_coef(double c, double h, int d, double omega) {
    double a = c / (h * h);
    double diag = 1.0 + 2.0 * d * a;
    return Coef<T>{T(a), T(diag), T(1.0 / diag), T(omega)};
}

#define ISDC_DISPATCH_D(d, ...)                      \
    switch (d) {                                     \
        case 1: { constexpr int D = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int D = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int D = 3; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;        \
    }

template <typename T>
hipError_t launch_smooth(const MGConfig& cfg, int n, const Coef<T>& co, bool zero_guess, const T* rhs,
                         const T* u_in, T* u_out, hipStream_t s) {
    const int d = cfg.d;
    if (cfg.smoother == ISDC_SMOOTH_JACOBI) {
        dim3 g = stencil_grid(d, n, n);
        ISDC_DISPATCH_D(d, {
            if (zero_guess)
                ISDC_GLAUNCH((k_jacobi<T, D, true>), g, dim3(kBlock), 0, s, rhs, u_in, u_out, n, co.a, co.diag, co.invdiag, co.w);
            else
                ISDC_GLAUNCH((k_jacobi<T, D, false>), g, dim3(kBlock), 0, s, rhs, u_in, u_out, n, co.a, co.diag, co.invdiag, co.w);
        });
        return hipGetLastError();
    }
    // RB-GS in place on u_out
    dim3 g = stencil_grid(d, (n + 1) / 2, n);
    ISDC_DISPATCH_D(d, {
        if (zero_guess)
            ISDC_GLAUNCH((k_rbgs_half<T, D, true>), g, dim3(kBlock), 0, s, rhs, u_out, n, co.a, co.invdiag, 0);
        else
            ISDC_GLAUNCH((k_rbgs_half<T, D, false>), g, dim3(kBlock), 0, s, rhs, u_out, n, co.a, co.invdiag, 0);
        ISDC_GLAUNCH((k_rbgs_half<T, D, false>), g, dim3(kBlock), 0, s, rhs, u_out, n, co.a, co.invdiag, 1);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int d, int n, const Coef<T>& co, const T* rhs, const T* u, T* rc, hipStream_t s) {
    int nc = (n - 1) / 2;
    dim3 g = stencil_grid(d, nc, nc);
    ISDC_DISPATCH_D(d, { ISDC_GLAUNCH((k_restrict<T, D>), g, dim3(kBlock), 0, s, rhs, u, rc, n, co.a, co.diag); });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(int d, int n, const T* ec, T* u, hipStream_t s) {
    dim3 g = stencil_grid(d, n, n);
    ISDC_DISPATCH_D(d, { ISDC_GLAUNCH((k_prolong<T, D>), g, dim3(kBlock), 0, s, ec, u, n); });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_resnorm(int d, int n, const Coef<T>& co, const T* rhs, const T* u, double* partial,
                          int* nblocks, hipStream_t s) {
    size_t N = d == 1 ? (size_t)n : (d == 2 ? (size_t)n * n : (size_t)n * n * n);
    int nb = reduce_blocks(N);
    *nblocks = nb;
    ISDC_DISPATCH_D(d, { ISDC_GLAUNCH((k_resnorm<T, D>), dim3(nb), dim3(kBlock), 0, s, rhs, u, n, co.a, co.diag, partial); });
    return hipGetLastError();
}

hipError_t launch_reduce_max(const double* partial, int nblocks, double* out, hipStream_t s) {
    ISDC_LAUNCH(k_reduce_max, dim3(1), dim3(kBlock), 0, s, partial, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_gate_reset(int* gate, hipStream_t s) {
    ISDC_LAUNCH(k_gate_reset, dim3(1), dim3(64), 0, s, gate);
    return hipGetLastError();
}

hipError_t launch_reduce_gate(const double* partial, int nblocks, double tol, int limit, int count_cycle, int* gate,
                              double* res_out, hipStream_t s) {
    ISDC_LAUNCH(k_reduce_gate, dim3(1), dim3(kBlock), 0, s, partial, nblocks, tol, limit, count_cycle, gate, res_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, size_t count, T value, hipStream_t s) {
    if (count == 0) return hipSuccess;
    ISDC_GLAUNCH((k_fill<T>), dim3(reduce_blocks(count)), dim3(kBlock), 0, s, p, count, value);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(const T* src, T* dst, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    ISDC_GLAUNCH((k_copy<T>), dim3(reduce_blocks(count)), dim3(kBlock), 0, s, src, dst, count);
    return hipGetLastError();
}

#define ISDC_INST(T)                                                                                      \
    template Coef<T> make_coef<T>(double, double, int, double);                                          \
    template hipError_t launch_smooth<T>(const MGConfig&, int, const Coef<T>&, bool, const T*, const T*, T*, \
                                         hipStream_t);                                                    \
    template hipError_t launch_restrict<T>(int, int, const Coef<T>&, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_prolong<T>(int, int, const T*, T*, hipStream_t);                          \
    template hipError_t launch_resnorm<T>(int, int, const Coef<T>&, const T*, const T*, double*, int*,  \
                                          hipStream_t);                                                   \
    template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);                                      \
    template hipError_t launch_copy<T>(const T*, T*, size_t, hipStream_t);

ISDC_INST(float)
ISDC_INST(double)

}  // namespace isdc
