// Outer SDC kernels in float64: the node-to-node quadrature S*F of eq. (2)
// fused with the max-norm SDC residual of Sec. 3, the right-hand side of the
// implicit Euler system of eq. (4), and the node update.
#include <hip/hip_runtime.h>
#include <cmath>

#include "internal.h"
#include "tile_common.h"

namespace isdc {

namespace {

constexpr int kBlock = kThreads;

__device__ __forceinline__ double nanmax(double a, double b) {
    if (a != a) return a;
    if (b != b) return b;
    return a > b ? a : b;
}

__device__ double block_max(double v) {
    __shared__ double sh[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < kBlock / 64; ++i) v = nanmax(v, sh[i]);
    return v;
}

template <int D>
__device__ __forceinline__ double lap_sum(const double* __restrict__ u, int n, int x, int y, int z, size_t i,
                                          double c) {
    // sum of neighbours - 2d * centre (zero ghosts)
    double s = -2.0 * D * c;
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

__device__ __forceinline__ double fexp(double u, int fe) { return fe == ISDC_FE_CUBIC ? u - u * u * u : 0.0; }

template <int D>
__device__ __forceinline__ void split(size_t i, int n, int& x, int& y, int& z) {
    // N < 2^31 for every admissible grid, so 32-bit division suffices
    const unsigned ii = (unsigned)i, un = (unsigned)n;
    x = (int)(ii % un);
    const unsigned t = ii / un;
    y = (D >= 2) ? (int)(t % un) : 0;
    z = (D == 3) ? (int)(t / un) : 0;
}

// Tiled form of the quadrature + residual kernel: one tile of points per
// workgroup, each node array staged in LDS (tile plus a halo of 1) in turn.
// Per point: f_j = nu L_h u_j + f^E(u_j); sf_m = sum_j dt s_{m,j} f_j;
// acc_m = u_0 + sum_j dt q_{m,j} f_j - u_m, and the tile's max |acc_m| goes
// to partial[workgroup].
template <int D, int M>
__global__ void __launch_bounds__(kThreads) k_quad_residual_tile(QuadArgs qa, int ntx, int nty, double* __restrict__ partial) {
    using B1 = HaloBox<D, 1>;
    using B0 = HaloBox<D, 0>;
    constexpr int P = B0::N / kThreads;
    __shared__ double su[B1::N];
    const int n = qa.n;
    int x0, y0, z0;
    tile_origin(ntx, nty, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    double sf[M][P], acc[M][P];
    bool ok[P];
    size_t gi[P];
    int li[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
        int lx, ly, lz;
        B0::split(threadIdx.x + kThreads * s, lx, ly, lz);
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        ok[s] = inside<D>(x, y, z, n);
        gi[s] = ok[s] ? gidx<D>(x, y, z, n) : 0;
        li[s] = ((lz + hz) * B1::Y + (ly + hy)) * B1::X + (lx + 1);
        const double u0 = ok[s] ? qa.u[0][gi[s]] : 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            sf[m][s] = 0.0;
            acc[m][s] = u0;
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j > 0) __syncthreads();
        stage<double, D, B1>(su, qa.u[j + 1], n, x0 - 1, y0 - hy, z0 - hz, false);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const double c = su[li[s]];
            const double f = qa.nu_h2 * (lds_nbsum<double, D, B1>(su, li[s]) - 2.0 * D * c) + fexp(c, qa.fe);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                sf[m][s] += qa.dtS[m * ISDC_MAX_M + j] * f;
                acc[m][s] += qa.dtQ[m * ISDC_MAX_M + j] * f;
            }
            acc[j][s] -= c;
        }
    }
    double mx = 0.0;
#pragma unroll
    for (int s = 0; s < P; ++s) {
        if (!ok[s]) continue;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (qa.sf[m]) qa.sf[m][gi[s]] = sf[m][s];
            mx = nanmax(mx, fabs(acc[m][s]));
        }
    }
    mx = block_max(mx);
    if (threadIdx.x == 0) partial[blockIdx.x] = mx;
}

// r = rhs - (I - c L_h) g, with
// rhs = u_m^{k+1} + dt_m [f^E(u_m^{k+1}) - f^E(u_m^k)] - dt_m nu L_h u_{m+1}^k + S F.
// For g = u_{m+1}^k the two L_h terms cancel and r is pointwise.
template <typename T, int D, int GUESS>
__global__ void __launch_bounds__(kBlock) k_euler_rhs(RhsArgs ra, T* __restrict__ r) {
    const int n = ra.n;
    const size_t N = (D == 1) ? (size_t)n : (D == 2 ? (size_t)n * n : (size_t)n * n * n);
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
        const double umn = ra.um_new[i], umo = ra.um_old[i], upo = ra.up_old[i];
        double base = umn + ra.dtm * (fexp(umn, ra.fe) - fexp(umo, ra.fe)) + ra.sf[i];
        double v;
        if (GUESS == ISDC_GUESS_PREV_SWEEP) {
            v = base - upo;
        } else {
            int x, y, z;
            split<D>(i, n, x, y, z);
            double rhs = base - ra.dtm * ra.nu_h2 * lap_sum<D>(ra.up_old, n, x, y, z, i, upo);
            if (GUESS == ISDC_GUESS_ZERO) {
                v = rhs;
            } else {  // PREV_NODE: g = u_m^{k+1}
                double Ag = umn - ra.dtm * ra.nu_h2 * lap_sum<D>(ra.um_new, n, x, y, z, i, umn);
                v = rhs - Ag;
            }
        }
        r[i] = T(v);
    }
}

template <typename T, int GUESS>
__global__ void __launch_bounds__(kBlock)
k_node_update(size_t N, const double* __restrict__ up_old, const double* __restrict__ um_new,
              const T* __restrict__ e, double* __restrict__ u_out) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (size_t)gridDim.x * kBlock) {
        double g = GUESS == ISDC_GUESS_PREV_SWEEP ? up_old[i] : (GUESS == ISDC_GUESS_ZERO ? 0.0 : um_new[i]);
        u_out[i] = g + (double)e[i];
    }
}

inline int grid_for(size_t N, int cap) {
    size_t b = (N + kBlock - 1) / kBlock;
    return (int)(b < (size_t)cap ? b : (size_t)cap);
}

}  // namespace

#define ISDC_DISPATCH_D(d, ...)                              \
    switch (d) {                                             \
        case 1: { constexpr int D = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int D = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int D = 3; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                \
    }

int quad_partials(int d, int n) {
    int ntx = 0, nty = 0, nb = 0;
    if (d == 1) tile_counts<1>(n, Tile<1>::X, Tile<1>::Y, Tile<1>::Z, ntx, nty, nb);
    else if (d == 2) tile_counts<2>(n, Tile<2>::X, Tile<2>::Y, Tile<2>::Z, ntx, nty, nb);
    else tile_counts<3>(n, Tile<3>::X, Tile<3>::Y, Tile<3>::Z, ntx, nty, nb);
    return nb;
}

template <int D>
static hipError_t launch_quad_d(const QuadArgs& qa, double* partial, int* nblocks, hipStream_t s) {
    int ntx, nty, nb;
    tile_counts<D>(qa.n, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, ntx, nty, nb);
    *nblocks = nb;
    switch (qa.M) {
#define ISDC_QM(MM) \
    case MM: hipLaunchKernelGGL((k_quad_residual_tile<D, MM>), dim3(nb), dim3(kThreads), 0, s, qa, ntx, nty, partial); break;
        ISDC_QM(1) ISDC_QM(2) ISDC_QM(3) ISDC_QM(4) ISDC_QM(5) ISDC_QM(6) ISDC_QM(7) ISDC_QM(8) ISDC_QM(9)
#undef ISDC_QM
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_quad_residual(int d, const QuadArgs& qa, double* partial, int* nblocks, hipStream_t s) {
    if (d == 1) return launch_quad_d<1>(qa, partial, nblocks, s);
    if (d == 2) return launch_quad_d<2>(qa, partial, nblocks, s);
    if (d == 3) return launch_quad_d<3>(qa, partial, nblocks, s);
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_euler_rhs(int d, const RhsArgs& ra, T* r, hipStream_t s) {
    size_t N = d == 1 ? (size_t)ra.n : (d == 2 ? (size_t)ra.n * ra.n : (size_t)ra.n * ra.n * ra.n);
    int nb = grid_for(N, 1 << 16);
    ISDC_DISPATCH_D(d, {
        switch (ra.guess) {
            case ISDC_GUESS_PREV_SWEEP:
                hipLaunchKernelGGL((k_euler_rhs<T, D, ISDC_GUESS_PREV_SWEEP>), dim3(nb), dim3(kBlock), 0, s, ra, r);
                break;
            case ISDC_GUESS_ZERO:
                hipLaunchKernelGGL((k_euler_rhs<T, D, ISDC_GUESS_ZERO>), dim3(nb), dim3(kBlock), 0, s, ra, r);
                break;
            default:
                hipLaunchKernelGGL((k_euler_rhs<T, D, ISDC_GUESS_PREV_NODE>), dim3(nb), dim3(kBlock), 0, s, ra, r);
                break;
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_node_update(size_t N, int guess, const double* up_old, const double* um_new, const T* e,
                              double* u_out, hipStream_t s) {
    int nb = grid_for(N, 1 << 16);
    switch (guess) {
        case ISDC_GUESS_PREV_SWEEP:
            hipLaunchKernelGGL((k_node_update<T, ISDC_GUESS_PREV_SWEEP>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
        case ISDC_GUESS_ZERO:
            hipLaunchKernelGGL((k_node_update<T, ISDC_GUESS_ZERO>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
        default:
            hipLaunchKernelGGL((k_node_update<T, ISDC_GUESS_PREV_NODE>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
    }
    return hipGetLastError();
}

template hipError_t launch_euler_rhs<float>(int, const RhsArgs&, float*, hipStream_t);
template hipError_t launch_euler_rhs<double>(int, const RhsArgs&, double*, hipStream_t);
template hipError_t launch_node_update<float>(size_t, int, const double*, const double*, const float*, double*, hipStream_t);
template hipError_t launch_node_update<double>(size_t, int, const double*, const double*, const double*, double*, hipStream_t);

}  // namespace isdc
