// Device bodies of the tiled multigrid kernels of 1D and 3D levels (see
// mg_tiles.hip for what each computes; 2D levels use rows2d.h) and the
// wave-level ordering of the single-workgroup tails.  A body works on one tile whose origin the
// caller supplies, so the same code serves the single-instance kernels (tile
// from the workgroup index) and the batched kernels (instance and tile from a
// table).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "tile_common.h"

namespace isdc {
namespace {

// Red update on the tile plus a halo of 1, then black on the tile, in LDS.
// se: box with halo 2 (origin tile - 2), sr: box with halo 1 (origin tile - 1).
// A colour's update reads only the other colour, so each is one lds_pass.
template <typename T, int D, class TL = Tile<D>>
__device__ __forceinline__ void rbgs_in_lds(T* se, const T* sr, int n, int x0, int y0, int z0, T a, T invdiag) {
    using B2 = HaloBoxT<D, 2, TL>;
    using B1 = HaloBoxT<D, 1, TL>;
    using B0 = HaloBoxT<D, 0, TL>;
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    lds_pass<T, B1>(se, [&](int k, int lx, int ly, int lz, T& v) {
        const int x = x0 - 1 + lx, y = y0 - hy + ly, z = z0 - hz + lz;
        if (!inside<D>(x, y, z, n) || ((x + y + z) & 1)) return -1;
        const int i = ((lz + hz) * B2::Y + (ly + hy)) * B2::X + (lx + 1);
        v = (sr[k] + a * lds_nbsum<T, D, B2>(se, i)) * invdiag;
        return i;
    });
    __syncthreads();
    lds_pass<T, B0>(se, [&](int, int lx, int ly, int lz, T& v) {
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside<D>(x, y, z, n) || !((x + y + z) & 1)) return -1;
        const int i = ((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2);
        const int k1 = ((lz + hz) * B1::Y + (ly + hy)) * B1::X + (lx + 1);
        v = (sr[k1] + a * lds_nbsum<T, D, B2>(se, i)) * invdiag;
        return i;
    });
    __syncthreads();
}

template <typename T, int D, bool ZERO, class TL = Tile<D>>
__device__ __forceinline__ void rbgs_tile_body(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out,
                                               int n, int x0, int y0, int z0, T a, T invdiag) {
    using B2 = HaloBoxT<D, 2, TL>;
    using B1 = HaloBoxT<D, 1, TL>;
    using B0 = HaloBoxT<D, 0, TL>;
    __shared__ T se[B2::N];
    __shared__ T sr[B1::N];
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    {
        Staged<T, D, B2> le;
        Staged<T, D, B1> lr;
        le.load(e_in, n, x0 - 2, y0 - 2 * hy, z0 - 2 * hz, ZERO);
        lr.load(r, n, x0 - 1, y0 - hy, z0 - hz, false);
        le.store(se);
        lr.store(sr);
    }
    __syncthreads();
    rbgs_in_lds<T, D, TL>(se, sr, n, x0, y0, z0, a, invdiag);
    for_box<B0>([&](int, int lx, int ly, int lz) {
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (inside<D>(x, y, z, n))
            e_out[gidx<D>(x, y, z, n)] = se[((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2)];
    });
}

template <typename T, int D>
__device__ __forceinline__ void restrict_tile_body(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc,
                                                   int n, int X0, int Y0, int Z0, T a, T diag) {
    using C = CTile<D>;
    using FB = Box<D, 2 * C::X + 1, 2 * C::Y + 1, 2 * C::Z + 1>;  // fine points under the coarse tile
    using EB = Box<D, 2 * C::X + 3, 2 * C::Y + 3, 2 * C::Z + 3>;  // ... plus a halo of 1
    using CB = Box<D, C::X, C::Y, C::Z>;
    __shared__ T se[EB::N];
    __shared__ T sres[FB::N];
    const int nc = (n - 1) / 2;
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    const int fx = 2 * X0, fy = 2 * Y0 * hy, fz = 2 * Z0 * hz;  // fine origin of FB
    {
        Staged<T, D, EB> le;
        Staged<T, D, FB> lr;
        le.load(e, n, fx - 1, fy - hy, fz - hz, false);
        lr.load(r, n, fx, fy, fz, false);
        le.store(se);
        lr.store(sres);
    }
    __syncthreads();
    lds_pass<T, FB>(sres, [&](int k, int lx, int ly, int lz, T& v) {
        if (!inside<D>(fx + lx, fy + ly, fz + lz, n)) return -1;
        const int i = ((lz + hz) * EB::Y + (ly + hy)) * EB::X + (lx + 1);
        v = sres[k] - (diag * se[i] - a * lds_nbsum<T, D, EB>(se, i));
        return k;
    });
    __syncthreads();
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for_box<CB>([&](int, int cx, int cy, int cz) {
        const int X = X0 + cx, Y = Y0 + cy, Z = Z0 + cz;
        if (!inside<D>(X, Y, Z, nc)) return;
        T acc = T(0);
#pragma unroll
        for (int oz = 0; oz < (D == 3 ? 3 : 1); ++oz) {
#pragma unroll
            for (int oy = 0; oy < (D >= 2 ? 3 : 1); ++oy) {
                const int base = ((2 * cz + oz) * FB::Y + (2 * cy + oy)) * FB::X + 2 * cx;
                T row = w[0] * sres[base] + w[1] * sres[base + 1] + w[2] * sres[base + 2];
                T wyz = (D >= 2 ? w[oy] : T(1)) * (D == 3 ? w[oz] : T(1));
                acc += wyz * row;
            }
        }
        rc[gidx<D>(X, Y, Z, nc)] = acc;
    });
}

// One red-black step from e_in to e_out fused with the residual of the new
// iterate and its full-weighting restriction to rc.  The tile's new iterate
// is computed on the tile plus a halo of 1 (red on a halo of 2), so the
// residual is available on every fine point under the tile's coarse points.
template <typename T, int D, bool ZERO, class TL = Tile<D>>
__device__ __forceinline__ void rbgs_restrict_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                   T* __restrict__ e_out, T* __restrict__ rc, int n, int x0, int y0,
                                                   int z0, T a, T diag, T invdiag) {
    using EB = Box<D, TL::X + 7, TL::Y + 7, TL::Z + 7>;  // old iterate, origin tile - 3
    using RB = Box<D, TL::X + 5, TL::Y + 5, TL::Z + 5>;  // rhs (later residual), origin tile - 2
    using BB = Box<D, TL::X + 3, TL::Y + 3, TL::Z + 3>;  // black region, origin tile - 1
    using RP = Box<D, TL::X + 1, TL::Y + 1, TL::Z + 1>;  // residual region, origin tile
    using B0 = Box<D, TL::X, TL::Y, TL::Z>;
    constexpr int CX = TL::X / 2, CY = D >= 2 ? TL::Y / 2 : 1, CZ = D == 3 ? TL::Z / 2 : 1;
    using CB = Box<D, CX, CY, CZ>;
    __shared__ T se[EB::N];
    __shared__ T sr[RB::N];
    const int nc = (n - 1) / 2;
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    {
        Staged<T, D, EB> le;
        Staged<T, D, RB> lr;
        le.load(e_in, n, x0 - 3, y0 - 3 * hy, z0 - 3 * hz, ZERO);
        lr.load(r, n, x0 - 2, y0 - 2 * hy, z0 - 2 * hz, false);
        le.store(se);
        lr.store(sr);
    }
    __syncthreads();
    auto eidx = [&](int lx, int ly, int lz, int off) {  // EB index of a point given in a box with origin tile - off
        return ((lz + (3 - off) * hz) * EB::Y + (ly + (3 - off) * hy)) * EB::X + (lx + 3 - off);
    };
    lds_pass<T, RB>(se, [&](int k, int lx, int ly, int lz, T& v) {  // red on the halo-2 region
        const int x = x0 - 2 + lx, y = y0 - 2 * hy + ly, z = z0 - 2 * hz + lz;
        if (!inside<D>(x, y, z, n) || ((x + y + z) & 1)) return -1;
        const int i = eidx(lx, ly, lz, 2);
        v = (sr[k] + a * lds_nbsum<T, D, EB>(se, i)) * invdiag;
        return i;
    });
    __syncthreads();
    lds_pass<T, BB>(se, [&](int, int lx, int ly, int lz, T& v) {  // black on the halo-1 region
        const int x = x0 - 1 + lx, y = y0 - hy + ly, z = z0 - hz + lz;
        if (!inside<D>(x, y, z, n) || !((x + y + z) & 1)) return -1;
        const int i = eidx(lx, ly, lz, 1);
        const int kr = ((lz + hz) * RB::Y + (ly + hy)) * RB::X + (lx + 1);
        v = (sr[kr] + a * lds_nbsum<T, D, EB>(se, i)) * invdiag;
        return i;
    });
    __syncthreads();
    for_box<B0>([&](int, int lx, int ly, int lz) {
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (inside<D>(x, y, z, n)) e_out[gidx<D>(x, y, z, n)] = se[eidx(lx, ly, lz, 0)];
    });
    lds_pass<T, RP>(sr, [&](int, int lx, int ly, int lz, T& v) {  // residual, in place of the rhs
        if (!inside<D>(x0 + lx, y0 + ly, z0 + lz, n)) return -1;
        const int i = eidx(lx, ly, lz, 0);
        const int kr = ((lz + 2 * hz) * RB::Y + (ly + 2 * hy)) * RB::X + (lx + 2);
        v = sr[kr] - (diag * se[i] - a * lds_nbsum<T, D, EB>(se, i));
        return kr;
    });
    __syncthreads();
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for_box<CB>([&](int, int cx, int cy, int cz) {
        const int X = x0 / 2 + cx, Y = (y0 / 2 + cy) * hy, Z = (z0 / 2 + cz) * hz;
        if (!inside<D>(X, Y, Z, nc)) return;
        T acc = T(0);
#pragma unroll
        for (int oz = 0; oz < (D == 3 ? 3 : 1); ++oz) {
#pragma unroll
            for (int oy = 0; oy < (D >= 2 ? 3 : 1); ++oy) {
                const int base = ((2 * cz + oz + 2 * hz) * RB::Y + (2 * cy + oy + 2 * hy)) * RB::X + 2 * cx + 2;
                T row = w[0] * sr[base] + w[1] * sr[base + 1] + w[2] * sr[base + 2];
                T wyz = (D >= 2 ? w[oy] : T(1)) * (D == 3 ? w[oz] : T(1));
                acc += wyz * row;
            }
        }
        rc[gidx<D>(X, Y, Z, nc)] = acc;
    });
}

template <typename T, int D, int MODE, class TL = Tile<D>>
__device__ __forceinline__ void prolong_rbgs_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                  const T* __restrict__ ec, T* __restrict__ e_out, int n, int x0, int y0,
                                                  int z0, T a, T invdiag, const double* __restrict__ g,
                                                  double* __restrict__ u_out) {
    using B2 = HaloBoxT<D, 2, TL>;
    using B1 = HaloBoxT<D, 1, TL>;
    using B0 = HaloBoxT<D, 0, TL>;
    using CB = Box<D, TL::X / 2 + 4, TL::Y / 2 + 4, TL::Z / 2 + 4>;
    __shared__ T se[B2::N];
    __shared__ T sr[B1::N];
    __shared__ T sc[CB::N];
    const int nc = (n - 1) / 2;
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    const int cxo = x0 / 2 - 2, cyo = (y0 / 2 - 2) * hy, czo = (z0 / 2 - 2) * hz;
    {
        Staged<T, D, B2> le;
        Staged<T, D, B1> lr;
        Staged<T, D, CB> lc;
        le.load(e_in, n, x0 - 2, y0 - 2 * hy, z0 - 2 * hz, false);
        lr.load(r, n, x0 - 1, y0 - hy, z0 - hz, false);
        lc.load(ec, nc, cxo, cyo, czo, false);
        le.store(se);
        lr.store(sr);
        lc.store(sc);
    }
    __syncthreads();
    // coarse-grid correction on the whole halo-2 box
    lds_pass<T, B2>(se, [&](int k, int lx, int ly, int lz, T& v) {
        const int x = x0 - 2 + lx, y = y0 - 2 * hy + ly, z = z0 - 2 * hz + lz;
        if (!inside<D>(x, y, z, n)) return -1;
        // linear interpolation per axis: odd index -> one coarse point, even
        // index -> mean of two; zeros outside [0, nc) are already staged
        int ix0, iy0 = 0, iz0 = 0;
        T wx1 = T(0), wy1 = T(0), wz1 = T(0), wx0 = T(1), wy0 = T(1), wz0 = T(1);
        if (x & 1) { ix0 = (x - 1) / 2 - cxo; }
        else { ix0 = x / 2 - 1 - cxo; wx0 = wx1 = T(0.5); }
        if (D >= 2) {
            if (y & 1) { iy0 = (y - 1) / 2 - cyo; }
            else { iy0 = y / 2 - 1 - cyo; wy0 = wy1 = T(0.5); }
        }
        if (D == 3) {
            if (z & 1) { iz0 = (z - 1) / 2 - czo; }
            else { iz0 = z / 2 - 1 - czo; wz0 = wz1 = T(0.5); }
        }
        // weights of the second tap are zero for odd indices, so reading it is harmless
        const int b00 = (iz0 * CB::Y + iy0) * CB::X + ix0;
        T acc = wy0 * (wx0 * sc[b00] + wx1 * sc[b00 + 1]);
        if (D >= 2) acc += wy1 * (wx0 * sc[b00 + CB::SY] + wx1 * sc[b00 + CB::SY + 1]);
        if (D == 3) {
            T acc1 = wy0 * (wx0 * sc[b00 + CB::SZ] + wx1 * sc[b00 + CB::SZ + 1]);
            acc1 += wy1 * (wx0 * sc[b00 + CB::SZ + CB::SY] + wx1 * sc[b00 + CB::SZ + CB::SY + 1]);
            acc = wz0 * acc + wz1 * acc1;
        }
        v = se[k] + acc;
        return k;
    });
    __syncthreads();
    rbgs_in_lds<T, D, TL>(se, sr, n, x0, y0, z0, a, invdiag);
    for_box<B0>([&](int, int lx, int ly, int lz) {
        const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside<D>(x, y, z, n)) return;
        const size_t gi = gidx<D>(x, y, z, n);
        const T v = se[((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2)];
        if (MODE == 0) e_out[gi] = v;
        else if (MODE == 1) u_out[gi] = g[gi] + (double)v;
        else u_out[gi] = (double)v;
    });
}

// ---------------------------------------------------------------- single-workgroup levels
// Threads of the single-workgroup coarse-tail kernels (tailc.h, ctail.h).
constexpr int kTail = 1024;

// Order the LDS accesses of one wave: the compiler keeps every access on its
// side of the fence, and the hardware executes one wave's LDS instructions in
// order, so what a lane stores before it is what any lane loads after it.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace
}  // namespace isdc
