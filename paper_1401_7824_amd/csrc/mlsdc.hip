// Grid transfers of two-level MLSDC (Sec. 5): the fine level has n = 2^k - 1
// interior points per axis, the coarse level n_c = (n - 1) / 2 (coarse point
// I on fine point 2I + 1, zero Dirichlet values at fine positions -1 and n).
//
//   * injection: coarse[I] = fine[2I + 1] per axis (node values and S F);
//   * the coarse correction u += P (uc_new - uc_old) with P the cubic
//     Lagrange interpolation per axis: an odd fine point copies its coarse
//     point; an even fine point 2I takes the cubic through the four known
//     values around it, the known values sitting at fine positions -1 (zero),
//     1, 3, ..., n - 2 (coarse) and n (zero), the four shifted inwards next
//     to the boundary (three points when n_c = 1).
//
// Both are one thread per fine (resp. coarse) point; they run once per node
// and MLSDC iteration, far from the V-cycles' share of the time.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace isdc {

namespace {

constexpr int kB = 256;

// Coarse taps of fine index i along one axis: count, coarse indices and
// weights (boundary taps, whose value is zero, are dropped).
struct Taps {
    int k;
    int idx[4];
    double w[4];
};

__device__ __forceinline__ Taps taps_of(int i, int nc) {
    Taps t;
    t.k = 0;
    if (i & 1) {
        t.k = 1;
        t.idx[0] = (i - 1) >> 1;
        t.w[0] = 1.0;
        return t;
    }
    const int I = i >> 1;  // between known points I and I + 1 (known index 0 = boundary -1)
    const int nk = nc + 2;  // known points: boundary, nc coarse, boundary
    const int cnt = nk < 4 ? nk : 4;
    int st = I - 1;
    if (st > nk - cnt) st = nk - cnt;
    if (st < 0) st = 0;
    const double x = (double)i;
    for (int a = st; a < st + cnt; ++a) {
        if (a == 0 || a == nk - 1) continue;  // zero boundary value
        const double pa = 2.0 * a - 1.0;
        double w = 1.0;
        for (int b = st; b < st + cnt; ++b)
            if (b != a) w *= (x - (2.0 * b - 1.0)) / (pa - (2.0 * b - 1.0));
        t.idx[t.k] = a - 1;
        t.w[t.k] = w;
        ++t.k;
    }
    return t;
}

template <int D>
__global__ void __launch_bounds__(kB) k_inject(const double* __restrict__ f, double* __restrict__ c, int n) {
    const int nc = (n - 1) / 2;
    const int X = blockIdx.x * kB + threadIdx.x;
    if (X >= nc) return;
    const int Y = D >= 2 ? (int)blockIdx.y : 0;
    const int Z = D == 3 ? (int)blockIdx.z : 0;
    const size_t fi = D == 1 ? (size_t)(2 * X + 1)
                    : D == 2 ? (size_t)(2 * Y + 1) * n + (2 * X + 1)
                             : ((size_t)(2 * Z + 1) * n + (2 * Y + 1)) * n + (2 * X + 1);
    const size_t ci = D == 1 ? (size_t)X : D == 2 ? (size_t)Y * nc + X : ((size_t)Z * nc + Y) * nc + X;
    c[ci] = f[fi];
}

template <int D>
__global__ void __launch_bounds__(kB)
k_cubic_correct(const double* __restrict__ cn, const double* __restrict__ co, double* __restrict__ u, int n) {
    const int nc = (n - 1) / 2;
    const int x = blockIdx.x * kB + threadIdx.x;
    if (x >= n) return;
    const int y = D >= 2 ? (int)blockIdx.y : 0;
    const int z = D == 3 ? (int)blockIdx.z : 0;
    const Taps tx = taps_of(x, nc);
    Taps ty, tz;
    ty.k = tz.k = 1;
    ty.idx[0] = tz.idx[0] = 0;
    ty.w[0] = tz.w[0] = 1.0;
    if (D >= 2) ty = taps_of(y, nc);
    if (D == 3) tz = taps_of(z, nc);
    double acc = 0.0;
    for (int c = 0; c < tz.k; ++c) {
        double accy = 0.0;
        for (int b = 0; b < ty.k; ++b) {
            const size_t row = ((size_t)tz.idx[c] * nc + ty.idx[b]) * nc;
            double accx = 0.0;
            for (int a = 0; a < tx.k; ++a) {
                const size_t j = row + tx.idx[a];
                accx += tx.w[a] * (cn[j] - co[j]);
            }
            accy += ty.w[b] * accx;
        }
        acc += tz.w[c] * accy;
    }
    const size_t i = D == 1 ? (size_t)x : D == 2 ? (size_t)y * n + x : ((size_t)z * n + y) * n + x;
    u[i] += acc;
}

dim3 grid_of(int d, int n) {
    return dim3((n + kB - 1) / kB, d >= 2 ? n : 1, d == 3 ? n : 1);
}

}  // namespace

hipError_t launch_inject(int d, int n, const double* fine, double* coarse, hipStream_t s) {
    const int nc = (n - 1) / 2;
    if (nc < 1) return hipErrorInvalidValue;
    const dim3 g = grid_of(d, nc);
    if (d == 1)
        hipLaunchKernelGGL(k_inject<1>, g, dim3(kB), 0, s, fine, coarse, n);
    else if (d == 2)
        hipLaunchKernelGGL(k_inject<2>, g, dim3(kB), 0, s, fine, coarse, n);
    else
        hipLaunchKernelGGL(k_inject<3>, g, dim3(kB), 0, s, fine, coarse, n);
    return hipGetLastError();
}

hipError_t launch_cubic_correct(int d, int n, const double* coarse_new, const double* coarse_old, double* u,
                                hipStream_t s) {
    if ((n - 1) / 2 < 1) return hipErrorInvalidValue;
    const dim3 g = grid_of(d, n);
    if (d == 1)
        hipLaunchKernelGGL(k_cubic_correct<1>, g, dim3(kB), 0, s, coarse_new, coarse_old, u, n);
    else if (d == 2)
        hipLaunchKernelGGL(k_cubic_correct<2>, g, dim3(kB), 0, s, coarse_new, coarse_old, u, n);
    else
        hipLaunchKernelGGL(k_cubic_correct<3>, g, dim3(kB), 0, s, coarse_new, coarse_old, u, n);
    return hipGetLastError();
}

}  // namespace isdc
