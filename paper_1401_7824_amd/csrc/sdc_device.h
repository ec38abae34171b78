// Device helpers of the outer SDC kernels (float64): NaN-propagating block
// maxima, the Laplacian stencil, f^E, and the body of the fused quadrature +
// SDC residual kernel, shared by the single-instance and batched kernels.
#pragma once

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

// The per-point arithmetic of the quadrature + residual kernels, shared by
// the tiled and the z-marched forms so both give the same bits:
// f_j = nu L_h u_j + f^E(u_j) from the centre c and the neighbour sum nb
// (x pair, then y pair, then z pair, as lds_nbsum adds them).
template <int D>
__device__ __forceinline__ double quad_f(double c, double nb, const QuadArgs& qa) {
    return qa.nu_h2 * (nb - 2.0 * D * c) + fexp(c, qa.fe);
}
template <int M>
__device__ __forceinline__ void quad_accumulate(double (&sf)[M], double (&acc)[M], double f, double c, int j,
                                                const QuadArgs& qa) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
        sf[m] += qa.dtS[m * ISDC_MAX_M + j] * f;
        acc[m] += qa.dtQ[m * ISDC_MAX_M + j] * f;
    }
    acc[j] -= c;
}

// Tiled form of the quadrature + residual kernel: one tile of points per
// workgroup, each node array staged in LDS (tile plus a halo of 1) in turn,
// the next two's loads in flight while the current one is used.
// Per point: f_j = nu L_h u_j + f^E(u_j); sf_m = sum_j dt s_{m,j} f_j;
// acc_m = u_0 + sum_j dt q_{m,j} f_j - u_m, and the tile's max |acc_m| goes
// to partial[workgroup].
// Returns the tile's max (valid in thread 0).
template <int D, int M>
__device__ __forceinline__ double quad_residual_body(const QuadArgs& qa, int x0, int y0, int z0) {
    using B1 = HaloBox<D, 1>;
    using B0 = HaloBox<D, 0>;
    constexpr int P = B0::N / kThreads;
    __shared__ double su[B1::N];
    const int n = qa.n;
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
    // the boxes of nodes j + 1 and j + 2 are loaded into registers while
    // node j is worked on (the node loop is unrolled, so each node's
    // registers are fixed and no load in flight is copied)
    constexpr int PD = M > 1 ? 2 : 1;
    Staged<double, D, B1> box[M];
#pragma unroll
    for (int j = 0; j < PD; ++j) box[j].load(qa.u[j + 1], n, x0 - 1, y0 - hy, z0 - hz, false);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        if (j > 0) __syncthreads();
        box[j].store(su);
        __syncthreads();
        if (j + PD < M) box[j + PD].load(qa.u[j + PD + 1], n, x0 - 1, y0 - hy, z0 - hz, false);
#pragma unroll
        for (int s = 0; s < P; ++s) {
            const double c = su[li[s]];
            const double f = quad_f<D>(c, lds_nbsum<double, D, B1>(su, li[s]), qa);
            double sfs[M], accs[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                sfs[m] = sf[m][s];
                accs[m] = acc[m][s];
            }
            quad_accumulate<M>(sfs, accs, f, c, j, qa);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                sf[m][s] = sfs[m];
                acc[m][s] = accs[m];
            }
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
    return block_max(mx);
}

}  // namespace
}  // namespace isdc
