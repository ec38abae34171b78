// 3D red-black Gauss-Seidel step by z-marching (device body).
//
// A 3D tile with a halo of 2 in every direction stages 3-5 times its own
// points; marching removes the z part of that overhead.  A workgroup owns an
// xy tile of MTile::X x MTile::Y points and a column of mz planes
// [z0, z0 + mz).  Planes of the iterate enter a ring of LDS planes (xy halo 2)
// as the march reaches them.  At step k the red points of plane k+1 are
// updated on the tile plus an xy halo of 1, then the black points of plane k
// on the tile; plane k is then final and goes to memory.  Red reads only old
// black values and black only new red values, so this is exactly one
// red-black step (red = even index sum, first).  Red on planes z0-1 and z0 is
// recomputed from the old iterate, so neighbouring columns never exchange
// data.  Every step first stores the planes loaded during the previous step
// into LDS and issues the loads for the next step, so global reads stay in
// flight while the step's LDS work runs.
//
// PRO: the iterate entering the ring is e_in + P e_c (trilinear
// interpolation of the coarse correction; coarse planes pass through one LDS
// buffer and their xy interpolation is kept in registers for the z weights).
// MODE as in the tiled body: 0 writes e_out, 1 writes the float64 node value
// g + e to u_out, 2 writes e to u_out (float64).  ZERO: e_in is zero.
#pragma once

#include <hip/hip_runtime.h>

#include "tile_common.h"

namespace isdc {
namespace {

struct MTile { static constexpr int X = 32, Y = 16; };

// Planes per marched column on an n^3 level, or 0 where the one-pass 3D tile
// kernels are used instead: a column costs a chain of Z + 4 dependent steps,
// which only pays where the level is large enough to fill the chip anyway.
// The tile shape of a marched level picks the depth: shape 0 the default,
// 1 twice as deep (fewer workgroups, less z overlap), 2 half as deep (more
// workgroups, shorter chains).  Every depth is even, so a column starts on an
// even plane, which the coarse-plane bookkeeping of the prolongation assumes.
__host__ __device__ constexpr int march_depth(int n, int shape = 0) {
    const int base = n >= 255 ? 16 : (n >= 127 ? 4 : 0);
    return shape == 1 ? 2 * base : (shape == 2 ? base / 2 : base);
}
static_assert(march_depth(127, 2) % 2 == 0 && march_depth(255, 2) % 2 == 0, "column depths are even");

template <typename T, bool PRO, int MODE, bool ZERO>
__device__ __forceinline__ void march_rbgs_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                const T* __restrict__ ec, T* __restrict__ e_out, int n, int x0, int y0,
                                                int z0, int mz, T a, T invdiag, const double* __restrict__ g,
                                                double* __restrict__ u_out) {
    using EP = Box<2, MTile::X + 4, MTile::Y + 4, 1>;          // iterate plane, origin (x0-2, y0-2)
    using RP = Box<2, MTile::X + 2, MTile::Y + 2, 1>;          // rhs plane, origin (x0-1, y0-1)
    using IP = Box<2, MTile::X, MTile::Y, 1>;                  // the tile
    using CP = Box<2, MTile::X / 2 + 4, MTile::Y / 2 + 4, 1>;  // coarse plane, origin (x0/2-2, y0/2-2)
    constexpr int NE = 5, NR = 3;                              // ring lengths (see the hazards below)
    constexpr int IE = (EP::N + kThreads - 1) / kThreads;
    constexpr int IR = (RP::N + kThreads - 1) / kThreads;
    constexpr int II = (IP::N + kThreads - 1) / kThreads;
    constexpr int IC = (CP::N + kThreads - 1) / kThreads;
    __shared__ T sE[NE][EP::N];
    __shared__ T sR[NR][RP::N];
    __shared__ T sC[PRO ? CP::N : 1];

    const size_t nn = (size_t)n * n;
    const int nc = (n - 1) / 2;
    const int z1 = min(z0 + mz, n);  // planes [z0, z1) are written
    const int cxo = x0 / 2 - 2, cyo = y0 / 2 - 2;
    auto ring = [](int p, int len) { return ((p % len) + len) % len; };

    T eraw[IE], rraw[IR], craw[IC], icur[IE];
    double graw[II];

    auto load_e = [&](int p) {
#pragma unroll
        for (int it = 0; it < IE; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            EP::split(k, lx, ly, lz);
            const int x = x0 - 2 + lx, y = y0 - 2 + ly;
            T v = T(0);
            if (!ZERO && k < EP::N && (unsigned)p < (unsigned)n && inside<2>(x, y, 0, n)) v = e_in[p * nn + (size_t)y * n + x];
            eraw[it] = v;
        }
    };
    auto load_r = [&](int p) {
#pragma unroll
        for (int it = 0; it < IR; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            RP::split(k, lx, ly, lz);
            const int x = x0 - 1 + lx, y = y0 - 1 + ly;
            T v = T(0);
            if (k < RP::N && (unsigned)p < (unsigned)n && inside<2>(x, y, 0, n)) v = r[p * nn + (size_t)y * n + x];
            rraw[it] = v;
        }
    };
    auto load_c = [&](int Z) {
#pragma unroll
        for (int it = 0; it < IC; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            CP::split(k, lx, ly, lz);
            const int X = cxo + lx, Y = cyo + ly;
            T v = T(0);
            if (k < CP::N && (unsigned)Z < (unsigned)nc && inside<2>(X, Y, 0, nc))
                v = ec[(size_t)Z * nc * nc + (size_t)Y * nc + X];
            craw[it] = v;
        }
    };
    auto store_c = [&]() {
#pragma unroll
        for (int it = 0; it < IC; ++it) {
            const int k = threadIdx.x + it * kThreads;
            if (k < CP::N) sC[k] = craw[it];
        }
    };
    // bilinear interpolation of the coarse plane in sC at this thread's
    // iterate-plane points (odd index: one coarse point, even: mean of two)
    auto interp_c = [&](T* out) {
#pragma unroll
        for (int it = 0; it < IE; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            EP::split(k, lx, ly, lz);
            const int x = x0 - 2 + lx, y = y0 - 2 + ly;
            T acc = T(0);
            if (k < EP::N && inside<2>(x, y, 0, n)) {
                int ix0, iy0;
                T wx1 = T(0), wy1 = T(0), wx0 = T(1), wy0 = T(1);
                if (x & 1) { ix0 = (x - 1) / 2 - cxo; }
                else { ix0 = x / 2 - 1 - cxo; wx0 = wx1 = T(0.5); }
                if (y & 1) { iy0 = (y - 1) / 2 - cyo; }
                else { iy0 = y / 2 - 1 - cyo; wy0 = wy1 = T(0.5); }
                const int b00 = iy0 * CP::X + ix0;
                acc = wy0 * (wx0 * sC[b00] + wx1 * sC[b00 + 1]);
                acc += wy1 * (wx0 * sC[b00 + CP::X] + wx1 * sC[b00 + CP::X + 1]);
            }
            out[it] = acc;
        }
    };

    // Prologue: coarse plane z0/2 - 2 gives the z-interpolation's first
    // operand; z0/2 - 1 waits in sC for the first even plane (z0 - 2).
    if (PRO) {
        load_c(z0 / 2 - 2);
        store_c();
        __syncthreads();
        interp_c(icur);
        __syncthreads();
        load_c(z0 / 2 - 1);
        store_c();
        __syncthreads();
    }
    load_e(z0 - 2);
    load_r(z0 - 3);

    // Step k stores plane k+2 of the iterate and k+1 of the rhs, then
    // updates red on k+1 and black on k.  Ring hazards: the store of plane
    // k+2 may overlap black(k-1) of slower threads, which reads k-2..k, so the
    // iterate ring needs 5 planes; the rhs store of k+1 may overlap their
    // read of rhs plane k-1, so that ring needs 3.
    for (int k = z0 - 4; k < z1; ++k) {
        const int pe = k + 2;  // iterate plane entering the ring
        T* se = sE[ring(pe, NE)];
        {
            T inew[IE];
            if (PRO && !(pe & 1)) interp_c(inew);  // coarse plane pe/2 (stored one step earlier)
#pragma unroll
            for (int it = 0; it < IE; ++it) {
                const int k2 = threadIdx.x + it * kThreads;
                if (k2 >= EP::N) break;
                T v = eraw[it];
                if (PRO) {
                    // odd plane: the coarse plane below; even: mean of the two around it
                    const T corr = (pe & 1) ? icur[it] : T(0.5) * icur[it] + T(0.5) * inew[it];
                    if ((unsigned)pe < (unsigned)n) v += corr;
                }
                se[k2] = v;
            }
            if (PRO && !(pe & 1)) {
#pragma unroll
                for (int it = 0; it < IE; ++it) icur[it] = inew[it];
            }
        }
        {
            T* sr = sR[ring(k + 1, NR)];
#pragma unroll
            for (int it = 0; it < IR; ++it) {
                const int k2 = threadIdx.x + it * kThreads;
                if (k2 < RP::N) sr[k2] = rraw[it];
            }
        }
        if (PRO && !((k + 3) & 1)) store_c();  // coarse plane (k+3)/2 for the next step
        // loads for the next step (and g of this step's output plane)
        load_e(k + 3);
        load_r(k + 2);
        if (PRO && !((k + 4) & 1)) load_c((k + 4) / 2);
        if (MODE == 1 && k >= z0) {
#pragma unroll
            for (int it = 0; it < II; ++it) {
                const int k2 = threadIdx.x + it * kThreads;
                int lx, ly, lz;
                IP::split(k2, lx, ly, lz);
                const int x = x0 + lx, y = y0 + ly;
                graw[it] = (k2 < IP::N && inside<2>(x, y, 0, n)) ? g[k * nn + (size_t)y * n + x] : 0.0;
            }
        }
        __syncthreads();
        // red on plane q = k+1, tile plus an xy halo of 1 (ghost planes
        // q < 0 and q >= n stay zero)
        const int q = k + 1;
        if (q >= z0 - 1 && q >= 0 && q < n) {
            T* em = sE[ring(q - 1, NE)];
            T* e0 = sE[ring(q, NE)];
            T* ep = sE[ring(q + 1, NE)];
            const T* sr = sR[ring(q, NR)];
            lds_pass<T, RP>(e0, [&](int kk, int lx, int ly, int, T& v) {
                const int x = x0 - 1 + lx, y = y0 - 1 + ly;
                if (!inside<2>(x, y, 0, n) || ((x + y + q) & 1)) return -1;
                const int i = (ly + 1) * EP::X + (lx + 1);
                const T nb = e0[i - 1] + e0[i + 1] + e0[i - EP::X] + e0[i + EP::X] + em[i] + ep[i];
                v = (sr[kk] + a * nb) * invdiag;
                return i;
            });
        }
        __syncthreads();
        // black on plane k, tile only; plane k is then final
        if (k >= z0) {
            T* em = sE[ring(k - 1, NE)];
            T* e0 = sE[ring(k, NE)];
            T* ep = sE[ring(k + 1, NE)];
            const T* sr = sR[ring(k, NR)];
#pragma unroll
            for (int it = 0; it < II; ++it) {
                const int k2 = threadIdx.x + it * kThreads;
                int lx, ly, lz;
                IP::split(k2, lx, ly, lz);
                const int x = x0 + lx, y = y0 + ly;
                if (k2 >= IP::N || !inside<2>(x, y, 0, n)) continue;
                const int i = (ly + 2) * EP::X + (lx + 2);
                T v = e0[i];
                if ((x + y + k) & 1) {
                    const int kr = (ly + 1) * RP::X + (lx + 1);
                    const T nb = e0[i - 1] + e0[i + 1] + e0[i - EP::X] + e0[i + EP::X] + em[i] + ep[i];
                    v = (sr[kr] + a * nb) * invdiag;
                }
                const size_t gi = k * nn + (size_t)y * n + x;
                if (MODE == 0) e_out[gi] = v;
                else if (MODE == 1) u_out[gi] = graw[it] + (double)v;
                else u_out[gi] = (double)v;
            }
        }
    }
}

// Residual r - A e of a 3D level and its full weighting onto the coarse
// level, z-marched.  A workgroup owns a coarse xy tile of MRTile::X x
// MRTile::Y points and a column of mzc coarse planes [Z0, Z0 + mzc).  Coarse
// plane Z takes the residual of fine planes 2Z, 2Z+1, 2Z+2 (coarse point I on
// fine 2I+1), and fine plane f needs the iterate on planes f-1..f+1: each step
// loads iterate planes 2Z+2, 2Z+3 (a ring of four, xy halo 1) and rhs planes
// 2Z+1, 2Z+2 (in registers, on the threads that compute the residual there),
// computes residual planes 2Z+1, 2Z+2 (a ring of three; 2Z is left from the
// step before) and writes coarse plane Z.  Each array is read about once
// instead of the 2-3 times of a 3D tile with a halo.  The residual and the
// weighted sums are the expressions of restrict_tile_body, term for term.
struct MRTile { static constexpr int X = 16, Y = 8; };
__host__ __device__ constexpr int march_restrict_depth() { return 8; }

template <typename T>
__device__ __forceinline__ void march_restrict_body(const T* __restrict__ r, const T* __restrict__ e,
                                                    T* __restrict__ rc, int n, int X0, int Y0, int Z0, int mzc, T a,
                                                    T diag) {
    using RB = Box<2, 2 * MRTile::X + 1, 2 * MRTile::Y + 1, 1>;  // residual plane, fine origin (2X0, 2Y0)
    using EB = Box<2, 2 * MRTile::X + 3, 2 * MRTile::Y + 3, 1>;  // iterate plane, origin (2X0-1, 2Y0-1)
    constexpr int IE = (EB::N + kThreads - 1) / kThreads;
    constexpr int IR = (RB::N + kThreads - 1) / kThreads;
    __shared__ T sE[4][EB::N];
    __shared__ T sRes[3][RB::N];
    const size_t nn = (size_t)n * n;
    const int nc = (n - 1) / 2;
    const int Z1 = min(Z0 + mzc, nc);
    const int fx = 2 * X0, fy = 2 * Y0;

    auto load_e = [&](T (&dst)[IE], int p) {
#pragma unroll
        for (int it = 0; it < IE; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            EB::split(k, lx, ly, lz);
            const int x = fx - 1 + lx, y = fy - 1 + ly;
            T v = T(0);
            if (k < EB::N && (unsigned)p < (unsigned)n && inside<2>(x, y, 0, n)) v = e[p * nn + (size_t)y * n + x];
            dst[it] = v;
        }
    };
    auto load_r = [&](T (&dst)[IR], int p) {
#pragma unroll
        for (int it = 0; it < IR; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            RB::split(k, lx, ly, lz);
            const int x = fx + lx, y = fy + ly;
            T v = T(0);
            if (k < RB::N && (unsigned)p < (unsigned)n && inside<2>(x, y, 0, n)) v = r[p * nn + (size_t)y * n + x];
            dst[it] = v;
        }
    };
    auto store_e = [&](const T (&src)[IE], int p) {
        T* d = sE[p & 3];
#pragma unroll
        for (int it = 0; it < IE; ++it) {
            const int k = threadIdx.x + it * kThreads;
            if (k < EB::N) d[k] = src[it];
        }
    };
    // residual of fine plane f (iterate planes f-1..f+1 in the ring) from the
    // thread's rhs values rr; points outside the grid keep 0
    auto residual = [&](const T (&rr)[IR], int f) {
        const T* em = sE[(f + 3) & 3];
        const T* e0 = sE[f & 3];
        const T* ep = sE[(f + 1) & 3];
        T* out = sRes[f % 3];
#pragma unroll
        for (int it = 0; it < IR; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            RB::split(k, lx, ly, lz);
            if (k >= RB::N) break;
            T v = T(0);
            if (inside<2>(fx + lx, fy + ly, 0, n)) {
                const int i = (ly + 1) * EB::X + (lx + 1);
                const T nb = e0[i - 1] + e0[i + 1] + e0[i - EB::X] + e0[i + EB::X] + em[i] + ep[i];
                v = rr[it] - (diag * e0[i] - a * nb);
            }
            out[k] = v;
        }
    };

    T ea[IE], eb[IE], ra[IR], rb[IR];
    // prologue: residual plane 2 Z0 from iterate planes 2Z0-1 .. 2Z0+1
    {
        const int f = 2 * Z0;
        load_e(ea, f - 1);
        load_e(eb, f);
        T ec[IE];
        load_e(ec, f + 1);
        load_r(ra, f);
        store_e(ea, f - 1);
        store_e(eb, f);
        store_e(ec, f + 1);
        __syncthreads();
        residual(ra, f);
        __syncthreads();  // the first step overwrites plane f - 1
    }
    // loads of the first step: iterate planes 2Z0+2, 2Z0+3, rhs 2Z0+1, 2Z0+2
    load_e(ea, 2 * Z0 + 2);
    load_e(eb, 2 * Z0 + 3);
    load_r(ra, 2 * Z0 + 1);
    load_r(rb, 2 * Z0 + 2);
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for (int Z = Z0; Z < Z1; ++Z) {
        const int f = 2 * Z;
        store_e(ea, f + 2);
        store_e(eb, f + 3);
        T rr1[IR], rr2[IR];
#pragma unroll
        for (int it = 0; it < IR; ++it) {
            rr1[it] = ra[it];
            rr2[it] = rb[it];
        }
        if (Z + 1 < Z1) {  // the next step's planes, in flight during this one
            load_e(ea, f + 4);
            load_e(eb, f + 5);
            load_r(ra, f + 3);
            load_r(rb, f + 4);
        }
        __syncthreads();
        residual(rr1, f + 1);
        residual(rr2, f + 2);
        __syncthreads();
        // coarse plane Z from residual planes f, f+1, f+2
        for (int c = threadIdx.x; c < MRTile::X * MRTile::Y; c += kThreads) {
            const int cx = c % MRTile::X, cy = c / MRTile::X;
            const int X = X0 + cx, Y = Y0 + cy;
            if (X >= nc || Y >= nc) continue;
            T acc = T(0);
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) {
                const T* s = sRes[(f + oz) % 3];
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    const int base = (2 * cy + oy) * RB::X + 2 * cx;
                    T row = w[0] * s[base] + w[1] * s[base + 1] + w[2] * s[base + 2];
                    T wyz = w[oy] * w[oz];
                    acc += wyz * row;
                }
            }
            rc[((size_t)Z * nc + Y) * nc + X] = acc;
        }
    }
}

}  // namespace
}  // namespace isdc
