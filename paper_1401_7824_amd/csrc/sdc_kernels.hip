// Outer SDC kernels in float64: the node-to-node quadrature S*F of eq. (2)
// fused with the max-norm SDC residual of Sec. 3, the right-hand side of the
// implicit Euler system of eq. (4), and the node update.
#include <hip/hip_runtime.h>
#include <cmath>

#include "internal.h"
#include "sdc_device.h"

namespace isdc {

namespace {

template <int D, int M>
__global__ void __launch_bounds__(kThreads) k_quad_residual_tile(QuadArgs qa, int ntx, int nty, double* __restrict__ partial) {
    int x0, y0, z0;
    tile_origin(ntx, nty, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
    const double mx = quad_residual_body<D, M>(qa, x0, y0, z0);
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
        // f^E = 0 (heat): u_m^k only enters through f^E, so it is not read
        const double umn = ra.um_new[i], umo = ra.fe == ISDC_FE_ZERO ? 0.0 : ra.um_old[i], upo = ra.up_old[i];
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
    case MM: ISDC_LAUNCH((k_quad_residual_tile<D, MM>), dim3(nb), dim3(kThreads), 0, s, qa, ntx, nty, partial); break;
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
                ISDC_LAUNCH((k_euler_rhs<T, D, ISDC_GUESS_PREV_SWEEP>), dim3(nb), dim3(kBlock), 0, s, ra, r);
                break;
            case ISDC_GUESS_ZERO:
                ISDC_LAUNCH((k_euler_rhs<T, D, ISDC_GUESS_ZERO>), dim3(nb), dim3(kBlock), 0, s, ra, r);
                break;
            default:
                ISDC_LAUNCH((k_euler_rhs<T, D, ISDC_GUESS_PREV_NODE>), dim3(nb), dim3(kBlock), 0, s, ra, r);
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
            ISDC_LAUNCH((k_node_update<T, ISDC_GUESS_PREV_SWEEP>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
        case ISDC_GUESS_ZERO:
            ISDC_LAUNCH((k_node_update<T, ISDC_GUESS_ZERO>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
        default:
            ISDC_LAUNCH((k_node_update<T, ISDC_GUESS_PREV_NODE>), dim3(nb), dim3(kBlock), 0, s, N, up_old, um_new, e, u_out);
            break;
    }
    return hipGetLastError();
}

template hipError_t launch_euler_rhs<float>(int, const RhsArgs&, float*, hipStream_t);
template hipError_t launch_euler_rhs<double>(int, const RhsArgs&, double*, hipStream_t);
template hipError_t launch_node_update<float>(size_t, int, const double*, const double*, const float*, double*, hipStream_t);
template hipError_t launch_node_update<double>(size_t, int, const double*, const double*, const double*, double*, hipStream_t);

}  // namespace isdc
