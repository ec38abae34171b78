// Row-mapped tiles of the fused weighted-Jacobi kernels of a 2D level
// (device bodies): K Jacobi steps fused with the residual's full weighting
// (cjres_tile), and the prolongation + correction fused with K Jacobi steps
// (cpjac_tile), for the compact nine-point operator B (C9) or the five-point
// operator I - c L_h, Dirichlet or periodic.  Used by the single-instance
// kernels and by the batch.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "tile_common.h"

namespace isdc {
namespace {

constexpr int kJL = 64;   // LDS columns (lanes per row)
constexpr int kJTY = 16;  // tile rows

// The two tiles of one compact V-cycle level, each on row-mapped tiles of
// TX x 16 points (64 LDS columns, one per lane), as device functions of the
// tile at (x0, y0) (the kernels k_cjres / k_cpjac and the batch kernels):
//   k_cjres  K Jacobi steps, then the residual r - B e on the fine points
//            under the tile's coarse points and its full weighting into rc;
//   k_cpjac  e + P e_c (linear interpolation) on the tile plus a halo of K,
//            then K Jacobi steps.
// The fine points of coarse point X are 2X + a (Dirichlet) or 2X - 1 + a
// (periodic), a = 0, 1, 2, so the residual region of a tile is x0 + sh ..
// x0 + sh + TX with sh = 0 / -1, the Jacobi steps run on it plus a halo of
// K - s + 1 at step s, and the staged box reaches K + 1 beyond it.  Every
// point gets the expressions of k_cjacobi, k_cresfw, k_prolong / k_cprolong_p.
template <int K> struct CVT {
    static constexpr int TX = (61 - 2 * K) & ~1, TY = kJTY;
    static constexpr int H = K + 1;                  // box halo around the residual region
    static constexpr int COLS = TX + 2 * H + 1, ROWS = TY + 2 * H + 1;
    static constexpr int RP = kThreads / kJL;
    static constexpr int IP = (ROWS + RP - 1) / RP;
    static constexpr int N = IP * kThreads;
    static_assert(COLS <= kJL, "box wider than a row of lanes");
};

// One weighted-Jacobi step of B from src to dst on LDS columns / rows
// [lo, chi] x [lo, rhi] of a box whose column c is grid x = bx + c, row q is
// y = by + q (Dirichlet: points outside the grid are not updated).
template <typename T, bool PER, int IP, bool ZERO, bool C9 = true>
__device__ __forceinline__ void cj_step(const T* src, T* dst, const T (&vr)[IP], int lo, int chi, int rhi, int bx,
                                        int by, int n, const CCoef<T>& k) {
    constexpr int L = kJL, RP = kThreads / kJL;
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    const int x = bx + c;
    const bool cok = c >= lo && c <= chi && (PER || (x >= 0 && x < n));
    T v[IP];
    bool wr[IP];
#pragma unroll
    for (int i = 0; i < IP; ++i) {
        const int q = j + i * RP;
        const int y = by + q;
        wr[i] = cok && q >= lo && q <= rhi && (PER || (y >= 0 && y < n));
        if (wr[i]) {
            const int a = threadIdx.x + i * kThreads;
            if (ZERO) {
                v[i] = k.omega * vr[i] * k.inv_b0;
            } else if (C9) {
                const T uc = src[a];
                const T edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                const T corners = src[a - L - 1] + src[a - L + 1] + src[a + L - 1] + src[a + L + 1];
                v[i] = uc + k.omega * (vr[i] - (k.b0 * uc + k.bf * edges + k.bc * corners)) * k.inv_b0;
            } else {
                const T uc = src[a];
                const T edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                v[i] = uc + k.omega * (vr[i] - (k.b0 * uc + k.bf * edges)) * k.inv_b0;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < IP; ++i)
        if (wr[i]) dst[threadIdx.x + i * kThreads] = v[i];
}

// Stage u over the box (column c: x = bx + c, row q: y = by + q; zero outside
// the grid or the box for Dirichlet, wrapped for periodic) into v.
template <typename T, bool PER, int IP>
__device__ __forceinline__ void cj_load(T (&v)[IP], const T* __restrict__ u, int bx, int by, int cols, int rows,
                                        int n) {
    constexpr int L = kJL, RP = kThreads / kJL;
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    int x = bx + c;
    if (PER) x = x < 0 ? x + n : (x >= n ? x - n : x);
    const bool xin = c < cols && (PER || (x >= 0 && x < n));
#pragma unroll
    for (int i = 0; i < IP; ++i) {
        const int q = j + i * RP;
        int y = by + q;
        if (PER) y = y < 0 ? y + n : (y >= n ? y - n : y);
        T val = T(0);
        if (xin && q < rows && (PER || (y >= 0 && y < n))) val = u[(size_t)y * n + x];
        v[i] = val;
    }
}

template <typename T, bool PER, int K, bool ZERO, bool C9 = true>
__device__ __forceinline__ void cjres_tile(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out,
                                           T* __restrict__ rc, int n, int x0, int y0, const CCoef<T>& k) {
    using V = CVT<K>;
    constexpr int L = kJL, H = V::H;
    __shared__ T sa[V::N];
    __shared__ T sb[V::N];
    constexpr int sh = PER ? -1 : 0;
    const int bx = x0 + sh - H, by = y0 + sh - H;  // grid point of LDS column / row 0
    T vr[V::IP];
    {
        T ve[V::IP];
        cj_load<T, PER>(vr, r, bx, by, V::COLS, V::ROWS, n);
        if (ZERO) {
#pragma unroll
            for (int i = 0; i < V::IP; ++i) ve[i] = T(0);
        } else {
            cj_load<T, PER>(ve, e_in, bx, by, V::COLS, V::ROWS, n);
        }
#pragma unroll
        for (int i = 0; i < V::IP; ++i) {
            sa[threadIdx.x + i * kThreads] = ve[i];
            sb[threadIdx.x + i * kThreads] = ve[i];
        }
    }
    __syncthreads();
    T* src = sa;
    T* dst = sb;
#pragma unroll
    for (int st = 1; st <= K; ++st) {
        if (ZERO && st == 1) cj_step<T, PER, V::IP, true, C9>(src, dst, vr, st, V::COLS - 1 - st, V::ROWS - 1 - st, bx, by, n, k);
        else cj_step<T, PER, V::IP, false, C9>(src, dst, vr, st, V::COLS - 1 - st, V::ROWS - 1 - st, bx, by, n, k);
        __syncthreads();
        T* t = src;
        src = dst;
        dst = t;
    }
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    {
        // the tile's points (columns / rows H - sh ..), then the residual on
        // columns / rows H .. H + TX (TY) into the free buffer
        const int x = bx + c;
        const bool tcol = c >= H - sh && c < H - sh + V::TX && x < n;
        const bool rcol = c >= H && c <= H + V::TX;
        T v[V::IP];
        bool wr[V::IP];
#pragma unroll
        for (int i = 0; i < V::IP; ++i) {
            const int q = j + i * V::RP;
            const int y = by + q;
            const int a = threadIdx.x + i * kThreads;
            if (tcol && q >= H - sh && q < H - sh + V::TY && y < n) e_out[(size_t)y * n + x] = src[a];
            wr[i] = rcol && q >= H && q <= H + V::TY;
            if (wr[i]) {
                const T uc = src[a];
                const T edges = src[a - 1] + src[a + 1] + src[a - L] + src[a + L];
                if (C9) {
                    const T corners = src[a - L - 1] + src[a - L + 1] + src[a + L - 1] + src[a + L + 1];
                    v[i] = vr[i] - (k.b0 * uc + k.bf * edges + k.bc * corners);
                } else {
                    v[i] = vr[i] - (k.b0 * uc + k.bf * edges);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < V::IP; ++i)
            if (wr[i]) dst[threadIdx.x + i * kThreads] = v[i];
    }
    __syncthreads();
    // full weighting: coarse (x0/2 + cx, y0/2 + cy) from columns / rows H + 2c + a
    const int nc = PER ? n / 2 : (n - 1) / 2;
    const int cx = threadIdx.x % (L / 2), cy0 = threadIdx.x / (L / 2);
    const int X = x0 / 2 + cx;
    if (cx >= V::TX / 2 || X >= nc) return;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
#pragma unroll
    for (int cy = cy0; cy < V::TY / 2; cy += 2 * kThreads / L) {
        const int Y = y0 / 2 + cy;
        if (Y >= nc) break;
        T acc = T(0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int base = (H + 2 * cy + b) * L + H + 2 * cx;
            T row = T(0);
#pragma unroll
            for (int a = 0; a < 3; ++a) row += w[a] * dst[base + a];
            acc += w[b] * row;
        }
        rc[(size_t)Y * nc + X] = acc;
    }
}

// MODE 0 writes the result to e_out; MODE 1 writes the float64 node value
// g + e to u_out instead (the last launch of an implicit solve).
template <typename T, bool PER, int K, bool C9 = true, int MODE = 0>
__device__ __forceinline__ void cpjac_tile(const T* __restrict__ r, const T* __restrict__ e_in,
                                           const T* __restrict__ ec, T* __restrict__ e_out, int n, int x0, int y0,
                                           const CCoef<T>& k, const double* __restrict__ g,
                                           double* __restrict__ u_out) {
    using V = CVT<K>;
    constexpr int L = kJL;
    constexpr int COLS = V::TX + 2 * K, ROWS = V::TY + 2 * K;
    __shared__ T sa[V::N];
    __shared__ T sb[V::N];
    const int bx = x0 - K, by = y0 - K;
    const int nc = PER ? n / 2 : (n - 1) / 2;
    T vr[V::IP];
    {
        T ve[V::IP];
        cj_load<T, PER>(vr, r, bx, by, COLS, ROWS, n);
        cj_load<T, PER>(ve, e_in, bx, by, COLS, ROWS, n);
        // e + P e_c at every staged point of the grid (coarse values from L2)
        const int c = threadIdx.x % L, j = threadIdx.x / L;
        int x = bx + c;
        if (PER) x = x < 0 ? x + n : (x >= n ? x - n : x);
        const bool xin = c < COLS && (PER || (x >= 0 && x < n));
#pragma unroll
        for (int i = 0; i < V::IP; ++i) {
            const int q = j + i * V::RP;
            int y = by + q;
            if (PER) y = y < 0 ? y + n : (y >= n ? y - n : y);
            if (xin && q < ROWS && (PER || (y >= 0 && y < n))) {
                T acc;
                if (PER) {
                    const int X0 = x >> 1, Y0 = y >> 1;
                    const int X1 = (x & 1) ? (X0 + 1 == nc ? 0 : X0 + 1) : X0;
                    const int Y1 = (y & 1) ? (Y0 + 1 == nc ? 0 : Y0 + 1) : Y0;
                    const T wx = (x & 1) ? T(0.5) : T(1), wy = (y & 1) ? T(0.5) : T(1);
                    const T wx1 = (x & 1) ? T(0.5) : T(0), wy1 = (y & 1) ? T(0.5) : T(0);
                    const T* r0 = ec + (size_t)Y0 * nc;
                    const T* r1 = ec + (size_t)Y1 * nc;
                    acc = wy * (wx * r0[X0] + wx1 * r0[X1]) + wy1 * (wx * r1[X0] + wx1 * r1[X1]);
                } else {
                    // taps of k_prolong (odd i -> (i-1)/2; even i -> i/2-1 and i/2
                    // inside [0, nc)), as two taps per axis whose weight is zero
                    // where k_prolong has none: every load issues at once, and a
                    // zero-weight term adds exactly nothing
                    const int ax = (x - 1) >> 1, ay = (y - 1) >> 1;  // first tap (odd: the only one)
                    const T wx0 = (x & 1) ? T(1) : (ax >= 0 ? T(0.5) : T(0));
                    const T wx1 = (x & 1) ? T(0) : (ax + 1 < nc ? T(0.5) : T(0));
                    const T wy0 = (y & 1) ? T(1) : (ay >= 0 ? T(0.5) : T(0));
                    const T wy1 = (y & 1) ? T(0) : (ay + 1 < nc ? T(0.5) : T(0));
                    const int X0 = max(ax, 0), X1 = min(ax + 1, nc - 1);
                    const int Y0 = max(ay, 0), Y1 = min(ay + 1, nc - 1);
                    const T* r0 = ec + (size_t)Y0 * nc;
                    const T* r1 = ec + (size_t)Y1 * nc;
                    const T c00 = r0[X0], c01 = r0[X1], c10 = r1[X0], c11 = r1[X1];
                    acc = T(0);
                    acc += wx0 * wy0 * T(1) * c00;
                    acc += wx1 * wy0 * T(1) * c01;
                    acc += wx0 * wy1 * T(1) * c10;
                    acc += wx1 * wy1 * T(1) * c11;
                }
                ve[i] += acc;
            }
        }
#pragma unroll
        for (int i = 0; i < V::IP; ++i) {
            sa[threadIdx.x + i * kThreads] = ve[i];
            sb[threadIdx.x + i * kThreads] = ve[i];
        }
    }
    __syncthreads();
    T* src = sa;
    T* dst = sb;
#pragma unroll
    for (int st = 1; st <= K; ++st) {
        cj_step<T, PER, V::IP, false, C9>(src, dst, vr, st, COLS - 1 - st, ROWS - 1 - st, bx, by, n, k);
        __syncthreads();
        T* t = src;
        src = dst;
        dst = t;
    }
    const int c = threadIdx.x % L, j = threadIdx.x / L;
    const int x = bx + c;
    if (c < K || c >= K + V::TX || x >= n) return;
#pragma unroll
    for (int i = 0; i < V::IP; ++i) {
        const int q = j + i * V::RP;
        const int y = by + q;
        if (q >= K && q < K + V::TY && y < n) {
            const size_t gi = (size_t)y * n + x;
            if (MODE == 0) e_out[gi] = src[threadIdx.x + i * kThreads];
            else u_out[gi] = g[gi] + (double)src[threadIdx.x + i * kThreads];
        }
    }
}

}  // namespace
}  // namespace isdc
