// 3D red-black Gauss-Seidel step by z-marching (device body).
//
// A 3D tile with a halo of 2 in every direction stages 3-5 times its own
// points; marching removes the z part of that overhead.  A workgroup owns an
// xy tile of MTile<T>::X x MTile<T>::Y points and a column of mz planes
// [z0, z0 + mz).  Planes of the iterate enter a ring of LDS planes (xy halo 2)
// as the march reaches them.  At step k the red points of plane k+1 are
// updated on the tile plus an xy halo of 1, then the black points of plane k
// on the tile; plane k is then final and goes to memory.  Red reads only old
// black values and black only new red values, so this is exactly one
// red-black step (red = even index sum, first).  Red on the planes just
// outside the column (z0 - 1 and z0 + mz) is recomputed from the old iterate,
// so neighbouring columns never exchange data.  Every step first stores the plane loaded during the previous step
// into LDS and issues the loads for the next step (the next plane of the
// iterate; the rhs at the next red and black points, which go to registers),
// so global reads stay in flight while the step's LDS work runs.
//
// PRO: the iterate entering the ring is e_in + P e_c (trilinear
// interpolation of the coarse correction; coarse planes pass through one LDS
// buffer and their xy interpolation is kept in registers for the z weights).
// MODE as in the tiled body: 0 writes e_out, 1 writes the float64 node value
// g + e to u_out, 2 writes e to u_out (float64).  ZERO: e_in is zero.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "tile_common.h"

namespace isdc {
namespace {

// Plane layout of the march (row-mapped, as the 2D row tiles): LPR = 64
// columns x0-2 .. x0+61 by ROWS = Y + 4 rows y0-2 .. y0+Y+1, stride LPR, for
// an xy tile of X = 60 by Y points (16 in float32, 8 in float64, so that a
// workgroup's ring of planes stays near 30 KB of LDS).  A plain pass (loads, LDS stores,
// the prolongation) gives thread t column t % LPR and rows t / LPR + RP i; a
// colour pass gives it colour lane t % H of rows t / H + RC i, and a row's
// H points of one colour sit one every other column, so every lane has a
// point of the colour and its column parity is fixed per plane.  LDS
// addresses are per-thread constants plus compile-time offsets, global ones a
// per-thread 32-bit byte offset from a uniform plane base.
template <int Y_>
struct MTileT {
    static constexpr int X = 60, Y = Y_;
    static constexpr int LPR = 64, ROWS = Y + 4;
    static constexpr int PN = LPR * ROWS;               // values per LDS plane
    static constexpr int RP = kThreads / LPR;           // rows per plain step
    static constexpr int IP = ROWS / RP;                // plain steps over a plane
    static constexpr int H = LPR / 2;                   // colour lanes per row
    static constexpr int RC = kThreads / H;             // rows per colour step
    static constexpr int IRED = (Y + 2 + RC - 1) / RC;  // red: rows 1 .. Y+2 (halo 1)
    static constexpr int IBLK = Y / RC;                 // black: rows 2 .. Y+1 (the tile)
    static constexpr int CROWS = Y / 2 + 4;             // coarse rows y0/2-2 .. (one spare)
    static constexpr int ICP = (CROWS + RP - 1) / RP;   // plain steps over the coarse plane
    static_assert(X + 4 == LPR && ROWS % RP == 0 && Y % RC == 0, "whole plain and colour steps");
    static_assert(RP % 2 == 0 && RC % 2 == 0 && X % 2 == 0, "even row steps keep a thread's row parity");
    static_assert(X / 2 + 4 <= LPR && ICP * RP >= CROWS, "the coarse plane fits the layout");
};
template <typename T>
using MTile = MTileT<sizeof(T) == 8 ? 8 : 16>;

// Planes per marched column on an n^3 level, or 0 where the one-pass 3D tile
// kernels are used instead: a column costs a chain of Z + 4 dependent steps,
// which only pays where the level is large enough to fill the chip anyway.
// The tile shape of a marched level picks the depth: shape 0 the default,
// 1 twice as deep (fewer workgroups, less z overlap; the single-instance
// launchers replace it by the depth that fits all columns in one round of
// resident workgroups), 2 half as deep (more workgroups, shorter chains).
// Every depth is even, so a column starts on an even plane, which the
// coarse-plane bookkeeping of the prolongation assumes.
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
    using M = MTile<T>;
    using TO = typename std::conditional<MODE == 0, T, double>::type;
    constexpr int L = M::LPR;
    // iterate ring: 5 planes, or 4 with one more barrier per step (see the
    // hazards below); the float64 prolongation kernels take 4, which brings
    // their LDS under 32 KB (five workgroups per CU); the plain step keeps 5
    // (measured: its extra barrier costs more than the occupancy gains)
    constexpr int NE = (PRO && sizeof(T) == 8) ? 4 : 5;
    __shared__ T sE[NE * M::PN];
    __shared__ T sC[PRO ? M::CROWS * L : 1];

    const size_t nn = (size_t)n * n;
    const int nc = (n - 1) / 2;
    const int z1 = min(z0 + mz, n);  // planes [z0, z1) are written
    // the domain 0 <= x, y < n in layout columns / rows (x = x0 - 2 + c, y = y0 - 2 + row)
    const int clo = max(0, 2 - x0), chi = min(L - 1, n + 1 - x0);
    const int rlo = max(0, 2 - y0), rhi = min(M::ROWS - 1, n + 1 - y0);
    const int rclo = max(1, clo), rchi = min(M::X + 2, chi), rrlo = max(1, rlo), rrhi = min(M::Y + 2, rhi);
    const int bclo = max(2, clo), bchi = min(M::X + 1, chi), brlo = max(2, rlo), brhi = min(M::Y + 1, rhi);
    const unsigned rowb = (unsigned)n * (unsigned)sizeof(T);
    const unsigned rowo = (unsigned)n * (unsigned)sizeof(TO);

    // plain mapping: column pc, rows pj + RP i
    const int pc = threadIdx.x % L, pj = threadIdx.x / L;
    const bool pcok = pc >= clo && pc <= chi;
    const unsigned poff = (unsigned)(y0 - 2 + pj) * rowb + (unsigned)(x0 - 2 + pc) * (unsigned)sizeof(T);
    // colour mapping: lane cl of rows cr + RC i; on plane p a row's points of
    // one colour have column parity cpar0 ^ (p & 1) (red rows start at row 1,
    // black rows at row 2: both give the same parity)
    const int cl = threadIdx.x % M::H, cr = threadIdx.x / M::H;
    const int cpar0 = (x0 + y0 + cr + 1) & 1;

    T eraw[M::IP], icur[M::IP];
    T rred[M::IRED], rblk[M::IBLK];          // rhs of this step's red and black points
    T rred_n[M::IRED], rblk_n[M::IBLK];      // ... and of the next step's
    double gb[M::IBLK][2], gb_n[M::IBLK][2];  // g at the black point and its red neighbour (MODE 1)
    T craw[M::ICP];

    auto load_e = [&](int p) {
        const bool pok = !ZERO && (unsigned)p < (unsigned)n;
        const T* b = pok ? e_in + (size_t)p * nn : e_in;
#pragma unroll
        for (int i = 0; i < M::IP; ++i) {
            const int row = pj + i * M::RP;
            T v = T(0);
            if (pok && pcok && row >= rlo && row <= rhi) v = at_byte(b, poff + (unsigned)(i * M::RP) * rowb);
            eraw[i] = v;
        }
    };
    // rhs at the red points of plane q (tile plus an xy halo of 1)
    auto load_rred = [&](int q) {
        const bool qok = q >= z0 - 1 && q >= 0 && q < n;
        const T* b = qok ? r + (size_t)q * nn : r;
        const int c = 2 * cl + (cpar0 ^ (q & 1));
        const bool cok = qok && c >= rclo && c <= rchi;
        const unsigned off = (unsigned)(y0 - 1 + cr) * rowb + (unsigned)(x0 - 2 + c) * (unsigned)sizeof(T);
#pragma unroll
        for (int i = 0; i < M::IRED; ++i) {
            const int row = 1 + cr + i * M::RC;
            T v = T(0);
            if (cok && row >= rrlo && row <= rrhi) v = at_byte(b, off + (unsigned)(i * M::RC) * rowb);
            rred_n[i] = v;
        }
    };
    // rhs at the black points of plane k (the tile), and g there and at the
    // red point beside each (MODE 1)
    auto load_rblk = [&](int k) {
        const bool kok = k >= z0 && k < z1;
        const T* b = kok ? r + (size_t)k * nn : r;
        const int par = cpar0 ^ (k & 1);
        const int cb = 2 * cl + par, cw = 2 * cl + (par ^ 1);
        const bool bok = kok && cb >= bclo && cb <= bchi, wok = kok && cw >= bclo && cw <= bchi;
        const unsigned off = (unsigned)(y0 + cr) * rowb + (unsigned)(x0 - 2 + cb) * (unsigned)sizeof(T);
#pragma unroll
        for (int i = 0; i < M::IBLK; ++i) {
            const int row = 2 + cr + i * M::RC;
            const bool rok = row >= brlo && row <= brhi;
            T v = T(0);
            if (bok && rok) v = at_byte(b, off + (unsigned)(i * M::RC) * rowb);
            rblk_n[i] = v;
            if (MODE == 1) {
                const double* gp = kok ? g + (size_t)k * nn : g;
                const unsigned rowg = (unsigned)n * 8u;
                const unsigned og = (unsigned)(y0 + cr + i * M::RC) * rowg;
                gb_n[i][0] = (bok && rok) ? at_byte(gp, og + (unsigned)(x0 - 2 + cb) * 8u) : 0.0;
                gb_n[i][1] = (wok && rok) ? at_byte(gp, og + (unsigned)(x0 - 2 + cw) * 8u) : 0.0;
            }
        }
    };
    // coarse plane Z, columns x0/2-2 .., rows y0/2-2 .. (zero outside 0 .. nc-1)
    auto load_c = [&](int Z) {
        const int X = x0 / 2 - 2 + pc;
        const bool ok = (unsigned)Z < (unsigned)nc && pc < M::X / 2 + 4 && X >= 0 && X < nc;
        const T* b = ok ? ec + (size_t)Z * nc * nc : ec;
        const unsigned rowc = (unsigned)nc * (unsigned)sizeof(T);
        const unsigned off = (unsigned)(y0 / 2 - 2 + pj) * rowc + (unsigned)X * (unsigned)sizeof(T);
#pragma unroll
        for (int i = 0; i < M::ICP; ++i) {
            const int Y = y0 / 2 - 2 + pj + i * M::RP;
            T v = T(0);
            if (ok && Y >= 0 && Y < nc) v = at_byte(b, off + (unsigned)(i * M::RP) * rowc);
            craw[i] = v;
        }
    };
    auto store_c = [&]() {
#pragma unroll
        for (int i = 0; i < M::ICP; ++i)
            if (pj + i * M::RP < M::CROWS) sC[threadIdx.x + i * kThreads] = craw[i];
    };
    // bilinear interpolation of the coarse plane in sC at this thread's plain
    // points (odd index: one coarse point, even: the mean of two; x0, y0 and
    // RP are even, so the parities are pc's and pj's)
    const T wx0 = (pc & 1) ? T(1) : T(0.5), wx1 = (pc & 1) ? T(0) : T(0.5);
    const T wy0 = (pj & 1) ? T(1) : T(0.5), wy1 = (pj & 1) ? T(0) : T(0.5);
    const int cb0 = ((pj + 1) >> 1) * L + ((pc + 1) >> 1);
    auto interp_c = [&](T* out) {
#pragma unroll
        for (int i = 0; i < M::IP; ++i) {
            const int row = pj + i * M::RP;
            T acc = T(0);
            if (pcok && row >= rlo && row <= rhi) {
                const int b = cb0 + i * (M::RP / 2) * L;
                acc = wy0 * (wx0 * sC[b] + wx1 * sC[b + 1]);
                acc += wy1 * (wx0 * sC[b + L] + wx1 * sC[b + L + 1]);
            }
            out[i] = acc;
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
#pragma unroll
    for (int i = 0; i < M::IRED; ++i) rred_n[i] = T(0);
#pragma unroll
    for (int i = 0; i < M::IBLK; ++i) {
        rblk_n[i] = T(0);
        gb_n[i][0] = gb_n[i][1] = 0.0;
    }

    // Step k stores plane k+2 of the iterate, then updates red on k+1 and
    // black on k.  Ring hazard: the store of plane k+2 may overlap black(k-1)
    // of slower threads, which reads planes k-2 .. k, so a ring of 5 slots
    // needs no barrier between steps; a ring of 4 (plane k+2 in the slot of
    // k-2) ends every step with one.  sk: the slot of plane k.
    int sk = ((z0 - 4) % NE + NE) % NE;
    auto slot = [&](int m) {  // slot of plane k + m, -1 <= m <= 2
        int v = sk + m;
        if (v >= NE) v -= NE;
        if (v < 0) v += NE;
        return v;
    };
    for (int k = z0 - 4; k < z1; ++k) {
#pragma unroll
        for (int i = 0; i < M::IRED; ++i) rred[i] = rred_n[i];
#pragma unroll
        for (int i = 0; i < M::IBLK; ++i) {
            rblk[i] = rblk_n[i];
            gb[i][0] = gb_n[i][0];
            gb[i][1] = gb_n[i][1];
        }
        const int pe = k + 2;  // iterate plane entering the ring
        {
            T* se = sE + slot(2) * M::PN;
            T inew[M::IP];
            if (PRO && !(pe & 1)) interp_c(inew);  // coarse plane pe/2 (stored one step earlier)
#pragma unroll
            for (int i = 0; i < M::IP; ++i) {
                T v = eraw[i];
                if (PRO) {
                    // odd plane: the coarse plane below; even: mean of the two around it
                    const T corr = (pe & 1) ? icur[i] : T(0.5) * icur[i] + T(0.5) * inew[i];
                    if ((unsigned)pe < (unsigned)n) v += corr;
                }
                se[threadIdx.x + i * kThreads] = v;
            }
            if (PRO && !(pe & 1)) {
#pragma unroll
                for (int i = 0; i < M::IP; ++i) icur[i] = inew[i];
            }
        }
        if (PRO && !((k + 3) & 1)) store_c();  // coarse plane (k+3)/2 for the next step
        // loads for the next step
        load_e(k + 3);
        load_rred(k + 2);
        load_rblk(k + 1);
        if (PRO && !((k + 4) & 1)) load_c((k + 4) / 2);
        __syncthreads();
        // red on plane q = k+1, tile plus an xy halo of 1 (ghost planes q < 0
        // and q >= n stay zero)
        const int q = k + 1;
        if (q >= z0 - 1 && q >= 0 && q < n) {
            const T* em = sE + slot(0) * M::PN;
            T* e0 = sE + slot(1) * M::PN;
            const T* ep = sE + slot(2) * M::PN;
            const int c = 2 * cl + (cpar0 ^ (q & 1));
            if (c >= rclo && c <= rchi) {
                T v[M::IRED];
                bool w[M::IRED];
#pragma unroll
                for (int i = 0; i < M::IRED; ++i) {
                    const int row = 1 + cr + i * M::RC;
                    w[i] = row >= rrlo && row <= rrhi;
                    if (w[i]) {
                        const int kk = row * L + c;
                        const T nb = e0[kk - 1] + e0[kk + 1] + e0[kk - L] + e0[kk + L] + em[kk] + ep[kk];
                        v[i] = (rred[i] + a * nb) * invdiag;
                    }
                }
#pragma unroll
                for (int i = 0; i < M::IRED; ++i)
                    if (w[i]) e0[(1 + cr + i * M::RC) * L + c] = v[i];
            }
        }
        __syncthreads();
        // black on plane k (the tile), written out with the red point beside
        // each: plane k is then final
        if (k >= z0) {
            const T* em = sE + slot(-1) * M::PN;
            const T* e0 = sE + slot(0) * M::PN;
            const T* ep = sE + slot(1) * M::PN;
            const int par = cpar0 ^ (k & 1);
            const int cb = 2 * cl + par, cw = 2 * cl + (par ^ 1);
            const bool bok = cb >= bclo && cb <= bchi, wok = cw >= bclo && cw <= bchi;
            TO* ob = MODE == 0 ? (TO*)e_out + (size_t)k * nn : (TO*)u_out + (size_t)k * nn;
            const unsigned ooff = (unsigned)(y0 + cr) * rowo;
#pragma unroll
            for (int i = 0; i < M::IBLK; ++i) {
                const int row = 2 + cr + i * M::RC;
                if (row < brlo || row > brhi) continue;
                const unsigned orow = ooff + (unsigned)(i * M::RC) * rowo;
                if (bok) {
                    const int kk = row * L + cb;
                    const T nb = e0[kk - 1] + e0[kk + 1] + e0[kk - L] + e0[kk + L] + em[kk] + ep[kk];
                    const T v = (rblk[i] + a * nb) * invdiag;
                    TO& o = at_byte(ob, orow + (unsigned)(x0 - 2 + cb) * (unsigned)sizeof(TO));
                    if (MODE == 0) o = (TO)v;
                    else if (MODE == 1) o = (TO)(gb[i][0] + (double)v);
                    else o = (TO)v;
                }
                if (wok) {
                    const T v = e0[row * L + cw];
                    TO& o = at_byte(ob, orow + (unsigned)(x0 - 2 + cw) * (unsigned)sizeof(TO));
                    if (MODE == 0) o = (TO)v;
                    else if (MODE == 1) o = (TO)(gb[i][1] + (double)v);
                    else o = (TO)v;
                }
            }
        }
        if (NE == 4) __syncthreads();  // black(k) has read plane k-1 before step k+1 stores k+3 there
        sk = sk == NE - 1 ? 0 : sk + 1;
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

// Zero-start red-black step fused with the residual and its full weighting,
// z-marched over the coarse planes of march_restrict_body's tile and column.
// From e = 0 one red-black step gives e = r / diag at the red points and
// e = (r + a * sum of the six red neighbours) / diag at the black ones, so the
// iterate is a function of r alone.  Each fine plane of r (xy halo 2) enters a
// ring of five LDS planes as r / diag at red points and r at black points;
// once the planes on either side are in, the black points of a plane (xy
// halo 1) are updated in place and the points the tile owns go to e_out.
// The residual of a fine plane (its rhs still in the registers that loaded
// it) goes to one of two LDS planes, and each coarse point's weighted sum
// is accumulated in a register over its three fine planes.  One pass over r
// replaces the zero-start step and the restriction: the iterate is written
// once and never read back.  The red value, the black neighbour sum and
// update, the residual and the weighted sums (added in the same order) are
// the expressions of the two kernels it replaces, term for term.
template <typename T>
__device__ __forceinline__ void march_zrestrict_body(const T* __restrict__ r, T* __restrict__ e_out,
                                                     T* __restrict__ rc, int n, int X0, int Y0, int Z0, int mzc, T a,
                                                     T diag, T invdiag) {
    using RB = Box<2, 2 * MRTile::X + 1, 2 * MRTile::Y + 1, 1>;  // residual plane, fine origin (2X0, 2Y0)
    using ZB = Box<2, 2 * MRTile::X + 5, 2 * MRTile::Y + 5, 1>;  // iterate plane, origin (2X0-2, 2Y0-2)
    constexpr int IZ = (ZB::N + kThreads - 1) / kThreads;
    constexpr int NS = 5;  // ring of fine planes f .. f+4 of a step
    constexpr int NC = MRTile::X * MRTile::Y;
    static_assert(NC <= kThreads, "one coarse point per thread");
    __shared__ T sZ[NS][ZB::N];
    __shared__ T sRes[2][RB::N];
    const size_t nn = (size_t)n * n;
    const int nc = (n - 1) / 2;
    const int Z1 = min(Z0 + mzc, nc);
    const int fx = 2 * X0, fy = 2 * Y0;
    auto slot = [](int p) { return (p % NS + NS) % NS; };

    // This thread's points of the plane box (the same in every pass): the
    // row offset in the level, the residual-box index, and flags: inside the
    // grid, in the black pass's box (halo 1), in the residual box, owned
    // (the tile writes fine columns [fx, fx + 2 X) and rows [fy, fy + 2 Y),
    // and column / row n - 1 where its coarse range reaches nc), and the
    // parity of x + y.
    enum { F_IN = 1, F_EB = 2, F_RB = 4, F_OWN = 8, F_ODD = 16 };
    unsigned goff[IZ];
    int rbi[IZ], fl[IZ];
#pragma unroll
    for (int it = 0; it < IZ; ++it) {
        const int k = threadIdx.x + it * kThreads;
        int lx, ly, lz;
        ZB::split(k, lx, ly, lz);
        const int x = fx - 2 + lx, y = fy - 2 + ly;
        int f = 0;
        if (k < ZB::N) {
            if (inside<2>(x, y, 0, n)) f |= F_IN;
            if (lx >= 1 && lx <= ZB::X - 2 && ly >= 1 && ly <= ZB::Y - 2) f |= F_EB;
            if (lx >= 2 && lx <= ZB::X - 3 && ly >= 2 && ly <= ZB::Y - 3) f |= F_RB;
            const bool ox = x >= fx && x < n && (x < fx + 2 * MRTile::X || x == n - 1);
            const bool oy = y >= fy && y < n && (y < fy + 2 * MRTile::Y || y == n - 1);
            if (ox && oy) f |= F_OWN;
            if ((lx + ly) & 1) f |= F_ODD;  // fx, fy even: the parity of x + y
        }
        fl[it] = f;
        goff[it] = (f & F_IN) ? (unsigned)y * (unsigned)n + (unsigned)x : 0u;
        rbi[it] = (ly - 2) * RB::X + (lx - 2);
    }

    auto load_z = [&](T (&dst)[IZ], int p) {
        const bool pok = (unsigned)p < (unsigned)n;
        const T* b = pok ? r + (size_t)p * nn : r;
#pragma unroll
        for (int it = 0; it < IZ; ++it) dst[it] = (pok && (fl[it] & F_IN)) ? b[goff[it]] : T(0);
    };
    // the value plane p holds at this thread's points when it enters the
    // ring: r / diag at red points (even x + y + p, final), r at black points
    // until their update
    auto entry = [&](const T (&src)[IZ], int p, T (&dst)[IZ]) {
#pragma unroll
        for (int it = 0; it < IZ; ++it) {
            const bool red = (((fl[it] & F_ODD) ? 1 : 0) + p) % 2 == 0;
            dst[it] = red ? src[it] * invdiag : src[it];
        }
    };
    auto store_z = [&](const T (&own)[IZ], int p) {
        T* d = sZ[slot(p)];
#pragma unroll
        for (int it = 0; it < IZ; ++it) {
            const int k = threadIdx.x + it * kThreads;
            if (k < ZB::N) d[k] = own[it];
        }
    };
    // A thread holds the same points k of every plane, and only it writes
    // them, so registers keep a copy of its own points of the middle ring
    // planes equal to the LDS plane at every pass: the centre and z
    // neighbours come from those registers (c for plane p, cm and cp for
    // p - 1 and p + 1; a null lm / lp takes that neighbour from the register,
    // else from that LDS plane), the four xy neighbours from LDS.
    // Black points of plane p (tile plus an xy halo of 1) from the red
    // values around them; the points the tile owns go to e_out.
    auto black = [&](int p, T (&c)[IZ], const T (&cm)[IZ], const T (&cp)[IZ], const T* lp) {
        if ((unsigned)p >= (unsigned)n) return;  // ghost planes stay zero
        T* e0 = sZ[slot(p)];
        const bool pown = p >= 2 * Z0 && (p < 2 * Z1 || p == n - 1);
        T* ob = e_out + (size_t)p * nn;
        const int pb = p & 1;
#pragma unroll
        for (int it = 0; it < IZ; ++it) {
            const int k = threadIdx.x + it * kThreads;
            if ((fl[it] & (F_EB | F_IN)) != (F_EB | F_IN)) continue;
            T v = c[it];
            if (((fl[it] & F_ODD) ? 1 : 0) != pb) {  // odd x + y + p
                const T up = lp ? lp[k] : cp[it];
                const T nb = e0[k - 1] + e0[k + 1] + e0[k - ZB::X] + e0[k + ZB::X] + cm[it] + up;
                v = (v + a * nb) * invdiag;
                e0[k] = v;
                c[it] = v;
            }
            if (pown && (fl[it] & F_OWN)) ob[goff[it]] = v;
        }
    };
    // residual of fine plane f (iterate planes f-1..f+1 in the ring) from
    // the rhs values rr this thread loaded for plane f; points outside the
    // grid keep 0
    auto residual = [&](const T (&rr)[IZ], int f, const T (&c)[IZ], const T (&cm)[IZ], const T (&cp)[IZ],
                        const T* lm) {
        const T* e0 = sZ[slot(f)];
        T* out = sRes[f & 1];
#pragma unroll
        for (int it = 0; it < IZ; ++it) {
            if (!(fl[it] & F_RB)) continue;
            const int i = threadIdx.x + it * kThreads;
            T v = T(0);
            if (fl[it] & F_IN) {
                const T dn = lm ? lm[i] : cm[it];
                const T nb = e0[i - 1] + e0[i + 1] + e0[i - ZB::X] + e0[i + ZB::X] + dn + cp[it];
                v = rr[it] - (diag * c[it] - a * nb);
            }
            out[rbi[it]] = v;
        }
    };
    // this thread's coarse point (threads below NC) and the weights
    const int cx = threadIdx.x % MRTile::X, cy = threadIdx.x / MRTile::X;
    const bool cown = threadIdx.x < NC && X0 + cx < nc && Y0 + cy < nc;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    // weighted rows of residual plane f with the z weight w[oz], added to acc
    auto weigh = [&](T& acc, int f, int oz) {
        const T* s = sRes[f & 1];
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const int base = (2 * cy + oy) * RB::X + 2 * cx;
            T row = w[0] * s[base] + w[1] * s[base + 1] + w[2] * s[base + 2];
            T wyz = w[oy] * w[oz];
            acc += wyz * row;
        }
    };
    auto copy = [](T (&d)[IZ], const T (&s)[IZ]) {
#pragma unroll
        for (int it = 0; it < IZ; ++it) d[it] = s[it];
    };

    // own iterate points of planes f+1 .. f+3 of a step in q1 .. q3
    T q1[IZ], q2[IZ], q3[IZ];
    T za[IZ], zb[IZ], r1[IZ], r2[IZ];
    T acc = T(0);
    const int f0 = 2 * Z0;
    // prologue: r planes f0-2 .. f0+2, iterate planes f0-1 .. f0+1, residual
    // plane f0 and its part of coarse plane Z0
    {
        T zc[IZ], m2[IZ], m1[IZ], q0[IZ];
        load_z(za, f0 - 2);
        load_z(zb, f0 - 1);
        load_z(zc, f0);
        load_z(r1, f0 + 1);
        load_z(r2, f0 + 2);
        entry(za, f0 - 2, m2);
        entry(zb, f0 - 1, m1);
        entry(zc, f0, q0);
        entry(r1, f0 + 1, q1);
        entry(r2, f0 + 2, q2);
        store_z(m2, f0 - 2);
        store_z(m1, f0 - 1);
        store_z(q0, f0);
        store_z(q1, f0 + 1);
        store_z(q2, f0 + 2);
        __syncthreads();
        // black(p) reads only red points of planes p-1 .. p+1, which no
        // black update writes: the three planes share one pass
        black(f0 - 1, m1, m2, q0, nullptr);
        black(f0, q0, m1, q1, nullptr);
        black(f0 + 1, q1, q0, q2, nullptr);
        __syncthreads();
        residual(zc, f0, q0, m1, q1, nullptr);
        __syncthreads();
        if (cown) weigh(acc, f0, 0);
    }
    // loads of the first step: r planes f0+3, f0+4
    load_z(za, f0 + 3);
    load_z(zb, f0 + 4);
    for (int Z = Z0; Z < Z1; ++Z) {
        const int f = 2 * Z;
        // planes f+3, f+4 go into the slots of f-2 and f-1, whose last
        // readers (the residuals of f-1 and f) passed the step's last barrier
        T n1[IZ], n2[IZ];
        copy(n1, za);
        copy(n2, zb);
        entry(n1, f + 3, q3);
        store_z(q3, f + 3);
        {
            T q4[IZ];
            entry(n2, f + 4, q4);
            store_z(q4, f + 4);
        }
        if (Z + 1 < Z1) {  // the next step's planes, in flight during this one
            load_z(za, f + 5);
            load_z(zb, f + 6);
        }
        __syncthreads();
        black(f + 2, q2, q1, q3, nullptr);
        black(f + 3, q3, q2, q3, sZ[slot(f + 4)]);
        __syncthreads();
        residual(r1, f + 1, q1, q1, q2, sZ[slot(f)]);
        residual(r2, f + 2, q2, q1, q3, nullptr);
        copy(r1, n1);
        copy(r2, n2);
        __syncthreads();
        // coarse plane Z from residual planes f (already in acc), f+1, f+2;
        // plane f+2 starts coarse plane Z+1
        if (cown) {
            weigh(acc, f + 1, 1);
            weigh(acc, f + 2, 2);
            rc[((size_t)Z * nc + (Y0 + cy)) * nc + (X0 + cx)] = acc;
            acc = T(0);
            weigh(acc, f + 2, 0);
        }
        // plane f+3 (its black points updated) and plane f+4 as it entered
        copy(q1, q3);
        entry(r2, f + 4, q2);
    }
}

// One red-black step from a nonzero iterate fused with the residual and its
// full weighting, z-marched over the coarse planes of march_restrict_body's
// tile and column.  Planes of the old iterate (xy halo 3) enter a ring of six
// LDS planes; per coarse step the red points of the two newest complete
// planes are updated on the tile plus an xy halo of 2 (they read only old
// black values: the black points of those planes are updated after them),
// then the black points of the two planes below on the tile plus a halo of
// 1 (reading only new red values), whose owned points go to e_out; the
// residual of the two planes below those goes to one of two LDS planes and
// each coarse point's weighted sum accumulates in a register.  The rhs of a
// plane stays in the registers that loaded it for its red, black and
// residual passes.  One pass replaces the red-black step and the
// restriction (the iterate is written once and never read back); the red
// and black updates, the residual and the weighted sums (added in the same
// order) are the expressions of the two kernels it replaces, term for term.
//
// A thread works on pairs of x-neighbours (even x, odd x): every pair has
// one point of each colour, so every lane has a point in each colour pass.
// An LDS plane holds its even columns, then its odd columns, each row-major
// with one value per pair, so a pass reads its neighbours at unit stride.  A
// thread holds the same pairs in every plane and only it writes them, so
// its registers keep a copy of its own points of the six ring planes equal
// to what LDS holds: the centre, the pair partner and the z neighbours come
// from registers, only the other x neighbour and the two y neighbours from
// LDS.
template <typename T>
__device__ __forceinline__ void march_srestrict_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                     T* __restrict__ e_out, T* __restrict__ rc, int n, int X0, int Y0,
                                                     int Z0, int mzc, T a, T diag, T invdiag) {
    using RB = Box<2, 2 * MRTile::X + 1, 2 * MRTile::Y + 1, 1>;  // residual plane, fine origin (2X0, 2Y0)
    constexpr int PX = MRTile::X + 4;      // pairs per row: fine columns 2X0-4 .. 2X0+2X+3
    constexpr int PR = 2 * MRTile::Y + 7;  // rows 2Y0-3 .. 2Y0+2Y+3
    constexpr int NP = PX * PR;            // pairs per plane
    constexpr int IP = (NP + kThreads - 1) / kThreads;
    constexpr int NS = 6;  // ring of fine planes f .. f+5 of a step
    constexpr int NC = MRTile::X * MRTile::Y;
    constexpr int OX = 2 * MRTile::X + 7;  // columns 2X0-3 .. 2X0+2X+3 hold the iterate (halo 3)
    static_assert(NC <= kThreads, "one coarse point per thread");
    __shared__ T sE[NS][2 * NP];  // [0, NP): even columns, [NP, 2 NP): odd columns
    __shared__ T sRes[2][RB::N];
    const size_t nn = (size_t)n * n;
    const int nc = (n - 1) / 2;
    const int Z1 = min(Z0 + mzc, nc);
    const int fx = 2 * X0, fy = 2 * Y0;
    auto slot = [](int p) { return (p % NS + NS) % NS; };

    // This thread's pairs (the same in every pass): the even point's offset
    // in a plane, the pair's row and index in an LDS half, the residual-box
    // index of its even point, and per point (even in bits 0-7, odd in bits
    // 8-15) flags: inside the grid; in the iterate box (halo 3), the red box
    // (halo 2), the black box (halo 1) or the residual box; owned.
    // Pairs are dealt out even rows first, then odd rows, so that most waves
    // hold rows of one parity, whose colour passes then take one branch.
    enum { F_IN = 1, F_OB = 2, F_ZB = 4, F_EB = 8, F_RB = 16, F_OWN = 32 };
    constexpr int NEVEN = (PR + 1) / 2 * PX;  // pairs in even rows
    unsigned goff[IP];
    int li[IP], rbi[IP], fl[IP], rowp[IP];
#pragma unroll
    for (int it = 0; it < IP; ++it) {
        const int k = threadIdx.x + it * kThreads;
        const int kk = k < NEVEN ? k : k - NEVEN;
        const int row = 2 * (kk / PX) + (k < NEVEN ? 0 : 1), j = kk % PX;
        const int x0 = fx - 4 + 2 * j, y = fy - 3 + row;
        int f = 0;
        if (k < NP) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int x = x0 + b, lx = 2 * j + b - 1;  // lx: column in the iterate box (origin 2X0-3)
                int g = 0;
                if (inside<2>(x, y, 0, n)) g |= F_IN;
                if (lx >= 0 && lx <= OX - 1) g |= F_OB;
                if (lx >= 1 && lx <= OX - 2 && row >= 1 && row <= PR - 2) g |= F_ZB;
                if (lx >= 2 && lx <= OX - 3 && row >= 2 && row <= PR - 3) g |= F_EB;
                if (lx >= 3 && lx <= OX - 4 && row >= 3 && row <= PR - 4) g |= F_RB;
                const bool ox = x >= fx && x < n && (x < fx + 2 * MRTile::X || x == n - 1);
                const bool oy = y >= fy && y < n && (y < fy + 2 * MRTile::Y || y == n - 1);
                if (ox && oy) g |= F_OWN;
                f |= g << (8 * b);
            }
        }
        fl[it] = f;
        // the odd point is inside only if the even one is (x0 is even)
        goff[it] = (f & F_IN) ? (unsigned)y * (unsigned)n + (unsigned)x0 : 0u;
        li[it] = k < NP ? row * PX + j : 0;
        rbi[it] = (row - 3) * RB::X + (x0 - fx);
        rowp[it] = row & 1;
    }
    auto has = [](int f, int b, int m) { return ((f >> (8 * b)) & m) == m; };

    // iterate plane p at this thread's points (zero outside the grid and the box)
    auto load_e = [&](T (&dst)[2 * IP], int p) {
        const bool pok = (unsigned)p < (unsigned)n;
        const T* bp = pok ? e_in + (size_t)p * nn : e_in;
#pragma unroll
        for (int it = 0; it < IP; ++it)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                dst[2 * it + b] = (pok && has(fl[it], b, F_IN | F_OB)) ? bp[goff[it] + b] : T(0);
    };
    // rhs of plane p at this thread's points of the red box
    auto load_r = [&](T (&dst)[2 * IP], int p) {
        const bool pok = (unsigned)p < (unsigned)n;
        const T* bp = pok ? r + (size_t)p * nn : r;
#pragma unroll
        for (int it = 0; it < IP; ++it)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                dst[2 * it + b] = (pok && has(fl[it], b, F_IN | F_ZB)) ? bp[goff[it] + b] : T(0);
    };
    auto store_e = [&](const T (&src)[2 * IP], int p) {
        T* d = sE[slot(p)];
#pragma unroll
        for (int it = 0; it < IP; ++it) {
            if (threadIdx.x + it * kThreads >= NP) continue;
            d[li[it]] = src[2 * it];
            d[NP + li[it]] = src[2 * it + 1];
        }
    };
    // One colour of plane p in place: red (even x + y + p) on the red box or
    // black on the black box; the black pass writes the owned points of p.
    // c: this thread's points of plane p, cm and cp: of p - 1 and p + 1.
    auto colour = [&](int p, const T (&rr)[2 * IP], bool blk, T (&c)[2 * IP], const T (&cm)[2 * IP],
                      const T (&cp)[2 * IP]) {
        if ((unsigned)p >= (unsigned)n) return;  // ghost planes stay zero
        T* e0 = sE[slot(p)];
        const bool pown = blk && p >= 2 * Z0 && (p < 2 * Z1 || p == n - 1);
        T* ob = e_out + (size_t)p * nn;
        const int box = (blk ? F_EB : F_ZB) | F_IN;
#pragma unroll
        for (int it = 0; it < IP; ++it) {
            const int l = li[it];
            // the even point is red when y + p is even (y = 2Y0 - 3 + row)
            const bool even_red = ((rowp[it] + 1 + p) & 1) == 0;
            if (blk != even_red) {  // the colour's point is the even one
                if (has(fl[it], 0, box)) {
                    const T nb = e0[NP + l - 1] + c[2 * it + 1] + e0[l - PX] + e0[l + PX] + cm[2 * it] + cp[2 * it];
                    const T v = (rr[2 * it] + a * nb) * invdiag;
                    e0[l] = v;
                    c[2 * it] = v;
                }
            } else if (has(fl[it], 1, box)) {  // ... the odd one
                const T nb = c[2 * it] + e0[l + 1] + e0[NP + l - PX] + e0[NP + l + PX] + cm[2 * it + 1] + cp[2 * it + 1];
                const T v = (rr[2 * it + 1] + a * nb) * invdiag;
                e0[NP + l] = v;
                c[2 * it + 1] = v;
            }
            if (pown) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    if (has(fl[it], b, F_OWN)) ob[goff[it] + b] = c[2 * it + b];
            }
        }
    };
    auto residual = [&](const T (&rr)[2 * IP], int f, const T (&c)[2 * IP], const T (&cm)[2 * IP],
                        const T (&cp)[2 * IP]) {
        const T* e0 = sE[slot(f)];
        T* out = sRes[f & 1];
#pragma unroll
        for (int it = 0; it < IP; ++it) {
            const int l = li[it];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (!has(fl[it], b, F_RB)) continue;
                T v = T(0);
                if (has(fl[it], b, F_IN)) {
                    const T xm = b == 0 ? e0[NP + l - 1] : c[2 * it];
                    const T xp = b == 0 ? c[2 * it + 1] : e0[l + 1];
                    const int yb = b == 0 ? l : NP + l;
                    const T nb = xm + xp + e0[yb - PX] + e0[yb + PX] + cm[2 * it + b] + cp[2 * it + b];
                    v = rr[2 * it + b] - (diag * c[2 * it + b] - a * nb);
                }
                out[rbi[it] + b] = v;
            }
        }
    };
    const int cx = threadIdx.x % MRTile::X, cy = threadIdx.x / MRTile::X;
    const bool cown = threadIdx.x < NC && X0 + cx < nc && Y0 + cy < nc;
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    auto weigh = [&](T& acc, int f, int oz) {
        const T* s = sRes[f & 1];
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const int base = (2 * cy + oy) * RB::X + 2 * cx;
            T row = w[0] * s[base] + w[1] * s[base + 1] + w[2] * s[base + 2];
            T wyz = w[oy] * w[oz];
            acc += wyz * row;
        }
    };
    auto copy = [](T (&d)[2 * IP], const T (&s)[2 * IP]) {
#pragma unroll
        for (int i = 0; i < 2 * IP; ++i) d[i] = s[i];
    };

    // own points of planes f .. f+5 of a step in q0 .. q5
    T q0[2 * IP], q1[2 * IP], q2[2 * IP], q3[2 * IP], q4[2 * IP], q5[2 * IP];
    T ea[2 * IP], eb[2 * IP], rA[2 * IP], rB[2 * IP], rC[2 * IP], rD[2 * IP];
    T acc = T(0);
    const int f0 = 2 * Z0;
    // prologue: red on planes f0-2 .. f0+2, black on f0-1 .. f0+1, residual
    // plane f0 and its part of coarse plane Z0
    {
        T m3[2 * IP], m2[2 * IP], m1[2 * IP], rr[2 * IP];
        // plane f0-3 is only a z neighbour (of red on f0-2): registers only
        load_e(m3, f0 - 3);
        load_e(m2, f0 - 2);
        load_e(m1, f0 - 1);
        load_e(q0, f0);
        load_e(q1, f0 + 1);
        load_e(q2, f0 + 2);
        load_e(q3, f0 + 3);
        load_r(rr, f0 - 2);
        load_r(rA, f0 - 1);
        load_r(rB, f0);
        load_r(rC, f0 + 1);
        load_r(rD, f0 + 2);
        store_e(m2, f0 - 2);
        store_e(m1, f0 - 1);
        store_e(q0, f0);
        store_e(q1, f0 + 1);
        store_e(q2, f0 + 2);
        store_e(q3, f0 + 3);
        __syncthreads();
        // a red pass reads only black points, which no red update writes:
        // the planes share one pass
        colour(f0 - 2, rr, false, m2, m3, m1);
        colour(f0 - 1, rA, false, m1, m2, q0);
        colour(f0, rB, false, q0, m1, q1);
        colour(f0 + 1, rC, false, q1, q0, q2);
        colour(f0 + 2, rD, false, q2, q1, q3);
        __syncthreads();
        colour(f0 - 1, rA, true, m1, m2, q0);
        colour(f0, rB, true, q0, m1, q1);
        colour(f0 + 1, rC, true, q1, q0, q2);
        __syncthreads();
        residual(rB, f0, q0, m1, q1);
        __syncthreads();
        if (cown) weigh(acc, f0, 0);
    }
    // registers of the first step: rhs of planes f0+1 .. f0+4 in rA .. rD,
    // iterate planes f0+4, f0+5 in ea, eb
    copy(rA, rC);
    copy(rB, rD);
    load_r(rC, f0 + 3);
    load_r(rD, f0 + 4);
    load_e(ea, f0 + 4);
    load_e(eb, f0 + 5);
    for (int Z = Z0; Z < Z1; ++Z) {
        const int f = 2 * Z;
        // planes f+4, f+5 go into the slots of f-2 and f-1, whose last
        // readers (the residuals of f-1 and f) passed the step's last barrier
        store_e(ea, f + 4);
        store_e(eb, f + 5);
        copy(q4, ea);
        copy(q5, eb);
        T rE[2 * IP], rF[2 * IP];
        if (Z + 1 < Z1) {  // the next step's planes, in flight during this one
            load_e(ea, f + 6);
            load_e(eb, f + 7);
            load_r(rE, f + 5);
            load_r(rF, f + 6);
        } else {
#pragma unroll
            for (int i = 0; i < 2 * IP; ++i) rE[i] = rF[i] = T(0);
        }
        __syncthreads();
        // red on f+3 and f+4 reads old black values of f+2 .. f+5
        colour(f + 3, rC, false, q3, q2, q4);
        colour(f + 4, rD, false, q4, q3, q5);
        __syncthreads();
        colour(f + 2, rB, true, q2, q1, q3);
        colour(f + 3, rC, true, q3, q2, q4);
        __syncthreads();
        residual(rA, f + 1, q1, q0, q2);
        residual(rB, f + 2, q2, q1, q3);
        __syncthreads();
        if (cown) {
            weigh(acc, f + 1, 1);
            weigh(acc, f + 2, 2);
            rc[((size_t)Z * nc + (Y0 + cy)) * nc + (X0 + cx)] = acc;
            acc = T(0);
            weigh(acc, f + 2, 0);
        }
        copy(rA, rC);
        copy(rB, rD);
        copy(rC, rE);
        copy(rD, rF);
        copy(q0, q2);
        copy(q1, q3);
        copy(q2, q4);
        copy(q3, q5);
    }
}

}  // namespace
}  // namespace isdc
