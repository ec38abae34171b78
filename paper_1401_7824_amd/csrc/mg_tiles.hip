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
//                       node array instead of e (the node update of eq. (4)).
//
// Workgroups are numbered so that each of the 8 XCDs (the hardware hands
// workgroup b to XCD b mod 8) receives a contiguous band of tiles, keeping the
// halo re-reads inside one XCD's L2.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace isdc {

namespace {

constexpr int kThreads = 256;

template <int D> struct Tile;
template <> struct Tile<1> { static constexpr int X = 1024, Y = 1, Z = 1; };
template <> struct Tile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 32, Y = 8, Z = 4; };

// Coarse tile of the restriction kernel.
template <int D> struct CTile;
template <> struct CTile<1> { static constexpr int X = 512, Y = 1, Z = 1; };
template <> struct CTile<2> { static constexpr int X = 32, Y = 8, Z = 1; };
template <> struct CTile<3> { static constexpr int X = 8, Y = 4, Z = 4; };

// A box of extents (X, Y, Z) in the used dimensions (unused ones are 1).
template <int D, int EX, int EY, int EZ>
struct Box {
    static constexpr int X = EX;
    static constexpr int Y = D >= 2 ? EY : 1;
    static constexpr int Z = D == 3 ? EZ : 1;
    static constexpr int N = X * Y * Z;
    static constexpr int SY = X;      // stride of y
    static constexpr int SZ = X * Y;  // stride of z
    __device__ static __forceinline__ void split(int k, int& lx, int& ly, int& lz) {
        lx = k % X;
        int t = k / X;
        ly = t % Y;
        lz = t / Y;
    }
};

template <int D, int H>
using HaloBox = Box<D, Tile<D>::X + 2 * H, Tile<D>::Y + 2 * H, Tile<D>::Z + 2 * H>;

template <int D>
__device__ __forceinline__ bool inside(int x, int y, int z, int n) {
    bool ok = (unsigned)x < (unsigned)n;
    if (D >= 2) ok = ok && (unsigned)y < (unsigned)n;
    if (D == 3) ok = ok && (unsigned)z < (unsigned)n;
    return ok;
}

template <int D>
__device__ __forceinline__ size_t gidx(int x, int y, int z, int n) {
    if (D == 1) return (size_t)x;
    if (D == 2) return (size_t)y * n + x;
    return ((size_t)z * n + y) * n + x;
}

// Logical tile of this workgroup: XCD k gets a contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, slot = b >> 3;
    return xcd * q + (xcd < rem ? xcd : rem) + slot;
}

__device__ __forceinline__ void tile_origin(int ntx, int nty, int TX, int TY, int TZ, int& x0, int& y0, int& z0) {
    int t = xcd_tile(blockIdx.x, gridDim.x);
    int tx = t % ntx;
    int r = t / ntx;
    int ty = r % nty;
    int tz = r / nty;
    x0 = tx * TX;
    y0 = ty * TY;
    z0 = tz * TZ;
}

// Sum of the 2d neighbours of LDS point i in box B (ghosts already zero).
template <typename T, int D, typename B>
__device__ __forceinline__ T lds_nbsum(const T* s, int i) {
    T v = s[i - 1] + s[i + 1];
    if (D >= 2) v += s[i - B::SY] + s[i + B::SY];
    if (D == 3) v += s[i - B::SZ] + s[i + B::SZ];
    return v;
}

// Stage a box of a global array whose origin is (ox, oy, oz); outside the
// domain the box holds zeros (homogeneous Dirichlet ghosts).
template <typename T, int D, typename B>
__device__ __forceinline__ void stage(T* s, const T* __restrict__ g, int n, int ox, int oy, int oz, bool zero) {
    for (int k = threadIdx.x; k < B::N; k += kThreads) {
        int lx, ly, lz;
        B::split(k, lx, ly, lz);
        int x = ox + lx, y = oy + ly, z = oz + lz;
        T v = T(0);
        if (!zero && inside<D>(x, y, z, n)) v = g[gidx<D>(x, y, z, n)];
        s[k] = v;
    }
}

// Red update on the tile plus a halo of 1, then black on the tile, in LDS.
// se: box with halo 2 (origin tile - 2), sr: box with halo 1 (origin tile - 1).
template <typename T, int D>
__device__ __forceinline__ void rbgs_in_lds(T* se, const T* sr, int n, int x0, int y0, int z0, T a, T invdiag) {
    using B2 = HaloBox<D, 2>;
    using B1 = HaloBox<D, 1>;
    using B0 = HaloBox<D, 0>;
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    for (int k = threadIdx.x; k < B1::N; k += kThreads) {
        int lx, ly, lz;
        B1::split(k, lx, ly, lz);
        int x = x0 - 1 + lx, y = y0 - hy + ly, z = z0 - hz + lz;
        if (!inside<D>(x, y, z, n) || ((x + y + z) & 1)) continue;
        int i = ((lz + hz) * B2::Y + (ly + hy)) * B2::X + (lx + 1);
        se[i] = (sr[k] + a * lds_nbsum<T, D, B2>(se, i)) * invdiag;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < B0::N; k += kThreads) {
        int lx, ly, lz;
        B0::split(k, lx, ly, lz);
        int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside<D>(x, y, z, n) || !((x + y + z) & 1)) continue;
        int i = ((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2);
        int k1 = ((lz + hz) * B1::Y + (ly + hy)) * B1::X + (lx + 1);
        se[i] = (sr[k1] + a * lds_nbsum<T, D, B2>(se, i)) * invdiag;
    }
    __syncthreads();
}

template <typename T, int D, bool ZERO>
__global__ void __launch_bounds__(kThreads)
k_rbgs_tile(const T* __restrict__ r, const T* __restrict__ e_in, T* __restrict__ e_out, int n, int ntx, int nty,
            T a, T invdiag) {
    using B2 = HaloBox<D, 2>;
    using B1 = HaloBox<D, 1>;
    using B0 = HaloBox<D, 0>;
    __shared__ T se[B2::N];
    __shared__ T sr[B1::N];
    int x0, y0, z0;
    tile_origin(ntx, nty, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    stage<T, D, B2>(se, e_in, n, x0 - 2, y0 - 2 * hy, z0 - 2 * hz, ZERO);
    stage<T, D, B1>(sr, r, n, x0 - 1, y0 - hy, z0 - hz, false);
    __syncthreads();
    rbgs_in_lds<T, D>(se, sr, n, x0, y0, z0, a, invdiag);
    for (int k = threadIdx.x; k < B0::N; k += kThreads) {
        int lx, ly, lz;
        B0::split(k, lx, ly, lz);
        int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside<D>(x, y, z, n)) continue;
        e_out[gidx<D>(x, y, z, n)] = se[((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2)];
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(kThreads)
k_restrict_tile(const T* __restrict__ r, const T* __restrict__ e, T* __restrict__ rc, int n, int ntx, int nty,
                T a, T diag) {
    using C = CTile<D>;
    using FB = Box<D, 2 * C::X + 1, 2 * C::Y + 1, 2 * C::Z + 1>;  // fine points under the coarse tile
    using EB = Box<D, 2 * C::X + 3, 2 * C::Y + 3, 2 * C::Z + 3>;  // ... plus a halo of 1
    __shared__ T se[EB::N];
    __shared__ T sres[FB::N];
    const int nc = (n - 1) / 2;
    int X0, Y0, Z0;
    tile_origin(ntx, nty, C::X, C::Y, C::Z, X0, Y0, Z0);
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    const int fx = 2 * X0, fy = 2 * Y0 * hy, fz = 2 * Z0 * hz;  // fine origin of FB
    stage<T, D, EB>(se, e, n, fx - 1, fy - hy, fz - hz, false);
    stage<T, D, FB>(sres, r, n, fx, fy, fz, false);
    __syncthreads();
    for (int k = threadIdx.x; k < FB::N; k += kThreads) {
        int lx, ly, lz;
        FB::split(k, lx, ly, lz);
        if (!inside<D>(fx + lx, fy + ly, fz + lz, n)) continue;
        int i = ((lz + hz) * EB::Y + (ly + hy)) * EB::X + (lx + 1);
        sres[k] = sres[k] - (diag * se[i] - a * lds_nbsum<T, D, EB>(se, i));
    }
    __syncthreads();
    const T w[3] = {T(0.25), T(0.5), T(0.25)};
    for (int k = threadIdx.x; k < C::X * (D >= 2 ? C::Y : 1) * (D == 3 ? C::Z : 1); k += kThreads) {
        int cx = k % C::X;
        int t = k / C::X;
        int cy = D >= 2 ? t % C::Y : 0;
        int cz = D == 3 ? t / C::Y : 0;
        int X = X0 + cx, Y = Y0 + cy, Z = Z0 + cz;
        if (!inside<D>(X, Y, Z, nc)) continue;
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
    }
}

template <typename T, int D, int MODE>
__global__ void __launch_bounds__(kThreads)
k_prolong_rbgs_tile(const T* __restrict__ r, const T* __restrict__ e_in, const T* __restrict__ ec, T* __restrict__ e_out,
                    int n, int ntx, int nty, T a, T invdiag, const double* __restrict__ g, double* __restrict__ u_out) {
    using B2 = HaloBox<D, 2>;
    using B1 = HaloBox<D, 1>;
    using B0 = HaloBox<D, 0>;
    using CB = Box<D, Tile<D>::X / 2 + 4, Tile<D>::Y / 2 + 4, Tile<D>::Z / 2 + 4>;
    __shared__ T se[B2::N];
    __shared__ T sr[B1::N];
    __shared__ T sc[CB::N];
    const int nc = (n - 1) / 2;
    int x0, y0, z0;
    tile_origin(ntx, nty, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, x0, y0, z0);
    const int hy = D >= 2 ? 1 : 0, hz = D == 3 ? 1 : 0;
    const int cxo = x0 / 2 - 2, cyo = (y0 / 2 - 2) * hy, czo = (z0 / 2 - 2) * hz;
    stage<T, D, B2>(se, e_in, n, x0 - 2, y0 - 2 * hy, z0 - 2 * hz, false);
    stage<T, D, B1>(sr, r, n, x0 - 1, y0 - hy, z0 - hz, false);
    stage<T, D, CB>(sc, ec, nc, cxo, cyo, czo, false);
    __syncthreads();
    // coarse-grid correction on the whole halo-2 box
    for (int k = threadIdx.x; k < B2::N; k += kThreads) {
        int lx, ly, lz;
        B2::split(k, lx, ly, lz);
        int x = x0 - 2 + lx, y = y0 - 2 * hy + ly, z = z0 - 2 * hz + lz;
        if (!inside<D>(x, y, z, n)) continue;
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
        se[k] += acc;
    }
    __syncthreads();
    rbgs_in_lds<T, D>(se, sr, n, x0, y0, z0, a, invdiag);
    for (int k = threadIdx.x; k < B0::N; k += kThreads) {
        int lx, ly, lz;
        B0::split(k, lx, ly, lz);
        int x = x0 + lx, y = y0 + ly, z = z0 + lz;
        if (!inside<D>(x, y, z, n)) continue;
        const size_t gi = gidx<D>(x, y, z, n);
        const T v = se[((lz + 2 * hz) * B2::Y + (ly + 2 * hy)) * B2::X + (lx + 2)];
        if (MODE == 0) e_out[gi] = v;
        else if (MODE == 1) u_out[gi] = g[gi] + (double)v;
        else u_out[gi] = (double)v;
    }
}

// ---------------------------------------------------------------- coarse tail
// All levels n_t, (n_t-1)/2, ..., 1 in one workgroup with every level's
// iterate, right-hand side and a residual scratch in LDS.  Threads are laid
// out as a fixed (x, y, z) block so that no index needs a division.

constexpr int kTail = 1024;
template <int D> struct TailLayout;
template <> struct TailLayout<1> { static constexpr int X = 1024, Y = 1, Z = 1, nmax = 2047, total = 4096; };
template <> struct TailLayout<2> { static constexpr int X = 64, Y = 16, Z = 1, nmax = 63, total = 5216; };
template <> struct TailLayout<3> { static constexpr int X = 16, Y = 16, Z = 4, nmax = 15, total = 3752; };

template <int D>
__device__ __forceinline__ int npts(int n) {
    return D == 1 ? n : (D == 2 ? n * n : n * n * n);
}

// Call f(x, y, z, i) for every point of an n^D level owned by this thread.
template <int D, typename F>
__device__ __forceinline__ void for_points(int n, F&& f) {
    using L = TailLayout<D>;
    const int tx = threadIdx.x % L::X;
    const int ty = (threadIdx.x / L::X) % L::Y;
    const int tz = threadIdx.x / (L::X * L::Y);
    for (int z = tz; z < (D == 3 ? n : 1); z += L::Z)
        for (int y = ty; y < (D >= 2 ? n : 1); y += L::Y)
            for (int x = tx; x < n; x += L::X) f(x, y, z, D == 1 ? x : (z * n + y) * n + x);
}

template <typename T, int D>
__device__ __forceinline__ T nb_lds(const T* e, int n, int x, int y, int z, int i) {
    T s = T(0);
    if (x > 0) s += e[i - 1];
    if (x < n - 1) s += e[i + 1];
    if (D >= 2) {
        if (y > 0) s += e[i - n];
        if (y < n - 1) s += e[i + n];
    }
    if (D == 3) {
        if (z > 0) s += e[i - n * n];
        if (z < n - 1) s += e[i + n * n];
    }
    return s;
}

template <typename T, int D>
__device__ void tail_smooth(T* e, const T* r, T* tmp, int n, T a, T diag, T invdiag, T w, int smoother) {
    if (smoother == ISDC_SMOOTH_RBGS) {
        for (int colour = 0; colour < 2; ++colour) {
            for_points<D>(n, [&](int x, int y, int z, int i) {
                if (((x + y + z) & 1) == colour) e[i] = (r[i] + a * nb_lds<T, D>(e, n, x, y, z, i)) * invdiag;
            });
            __syncthreads();
        }
    } else {
        for_points<D>(n, [&](int x, int y, int z, int i) {
            T c = e[i];
            tmp[i] = c + w * ((r[i] - (diag * c - a * nb_lds<T, D>(e, n, x, y, z, i))) * invdiag);
        });
        __syncthreads();
        for_points<D>(n, [&](int x, int y, int z, int i) { e[i] = tmp[i]; });
        __syncthreads();
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(kTail)
k_tail(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t, double c, double h_t, int smoother, int nu1,
       int nu2, double omega, int zero_guess) {
    using L = TailLayout<D>;
    __shared__ T le[L::total];
    __shared__ T lr[L::total];
    __shared__ T lt[D == 1 ? 2048 : (D == 2 ? 3969 : 3375)];
    int nlev = 0, off[16], nn[16];
    for (int o = 0, n = n_t;; n = (n - 1) / 2) {
        off[nlev] = o;
        nn[nlev] = n;
        o += npts<D>(n);
        ++nlev;
        if (n == 1) break;
    }
    {
        const int N0 = npts<D>(n_t);
        for (int i = threadIdx.x; i < N0; i += kTail) {
            lr[i] = rhs_g[i];
            le[i] = zero_guess ? T(0) : e_g[i];
        }
    }
    __syncthreads();
    const T wts[3] = {T(0.25), T(0.5), T(0.25)};
    double h = h_t;
    for (int l = 0; l < nlev; ++l) {
        const int n = nn[l];
        const double ad = c / (h * h);
        const T a = T(ad), diag = T(1.0 + 2.0 * D * ad), invdiag = T(1.0 / (1.0 + 2.0 * D * ad));
        T* e = le + off[l];
        T* r = lr + off[l];
        if (n == 1) {
            if (threadIdx.x == 0) e[0] = r[0] / diag;
            __syncthreads();
            break;
        }
        for (int k = 0; k < nu1; ++k) tail_smooth<T, D>(e, r, lt, n, a, diag, invdiag, T(omega), smoother);
        for_points<D>(n, [&](int x, int y, int z, int i) {
            lt[i] = r[i] - (diag * e[i] - a * nb_lds<T, D>(e, n, x, y, z, i));
        });
        __syncthreads();
        const int nc = (n - 1) / 2;
        T* rc = lr + off[l + 1];
        T* ec = le + off[l + 1];
        for_points<D>(nc, [&](int X, int Y, int Z, int I) {
            T acc = T(0);
            for (int oz = 0; oz < (D == 3 ? 3 : 1); ++oz)
                for (int oy = 0; oy < (D >= 2 ? 3 : 1); ++oy) {
                    const int fy = D >= 2 ? 2 * Y + oy : 0, fz = D == 3 ? 2 * Z + oz : 0;
                    const int base = (D == 1 ? 0 : (fz * n + fy) * n) + 2 * X;
                    T row = wts[0] * lt[base] + wts[1] * lt[base + 1] + wts[2] * lt[base + 2];
                    acc += (D >= 2 ? wts[oy] : T(1)) * (D == 3 ? wts[oz] : T(1)) * row;
                }
            rc[I] = acc;
            ec[I] = T(0);
        });
        __syncthreads();
        h *= 2.0;
    }
    for (int l = nlev - 2; l >= 0; --l) {
        h *= 0.5;
        const int n = nn[l];
        const int nc = nn[l + 1];
        const double ad = c / (h * h);
        const T a = T(ad), diag = T(1.0 + 2.0 * D * ad), invdiag = T(1.0 / (1.0 + 2.0 * D * ad));
        T* e = le + off[l];
        T* r = lr + off[l];
        const T* ec = le + off[l + 1];
        for_points<D>(n, [&](int x, int y, int z, int i) {
            // linear interpolation, one axis at a time: odd -> (i-1)/2, even -> mean of i/2-1, i/2
            int ix0, ix1, iy0 = 0, iy1 = 0, iz0 = 0, iz1 = 0;
            T wx0, wx1, wy0 = T(1), wy1 = T(0), wz0 = T(1), wz1 = T(0);
            if (x & 1) { ix0 = ix1 = (x - 1) / 2; wx0 = T(1); wx1 = T(0); }
            else { ix0 = x / 2 - 1; ix1 = x / 2; wx0 = wx1 = T(0.5); }
            if (D >= 2) {
                if (y & 1) { iy0 = iy1 = (y - 1) / 2; }
                else { iy0 = y / 2 - 1; iy1 = y / 2; wy0 = wy1 = T(0.5); }
            }
            if (D == 3) {
                if (z & 1) { iz0 = iz1 = (z - 1) / 2; }
                else { iz0 = z / 2 - 1; iz1 = z / 2; wz0 = wz1 = T(0.5); }
            }
            auto at = [&](int X, int Y, int Z) -> T {
                if (X < 0 || X >= nc) return T(0);
                if (D >= 2 && (Y < 0 || Y >= nc)) return T(0);
                if (D == 3 && (Z < 0 || Z >= nc)) return T(0);
                return ec[(D == 1) ? X : ((Z * nc + Y) * nc + X)];
            };
            T acc = T(0);
            const int nzt = D == 3 ? 2 : 1, nyt = D >= 2 ? 2 : 1;
            for (int cz = 0; cz < nzt; ++cz)
                for (int cy = 0; cy < nyt; ++cy) {
                    const int Y = cy ? iy1 : iy0, Z = cz ? iz1 : iz0;
                    const T wyz = (cy ? wy1 : wy0) * (cz ? wz1 : wz0);
                    if (wyz == T(0)) continue;
                    T row = wx0 * at(ix0, Y, Z);
                    if (wx1 != T(0)) row += wx1 * at(ix1, Y, Z);
                    acc += wyz * row;
                }
            e[i] += acc;
        });
        __syncthreads();
        for (int k = 0; k < nu2; ++k) tail_smooth<T, D>(e, r, lt, n, a, diag, invdiag, T(omega), smoother);
    }
    {
        const int N0 = npts<D>(n_t);
        for (int i = threadIdx.x; i < N0; i += kTail) e_g[i] = le[i];
    }
}

template <int D>
inline void tile_counts(int n, int TX, int TY, int TZ, int& ntx, int& nty, int& nb) {
    ntx = (n + TX - 1) / TX;
    nty = D >= 2 ? (n + TY - 1) / TY : 1;
    int ntz = D == 3 ? (n + TZ - 1) / TZ : 1;
    nb = ntx * nty * ntz;
}

}  // namespace

#define ISDC_DISPATCH_D(d, ...)                              \
    switch (d) {                                             \
        case 1: { constexpr int D = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int D = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int D = 3; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                \
    }

template <typename T>
hipError_t launch_rbgs_tile(int d, int n, const Coef<T>& co, bool zero, const T* r, const T* e_in, T* e_out,
                            hipStream_t s) {
    ISDC_DISPATCH_D(d, {
        int ntx, nty, nb;
        tile_counts<D>(n, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, ntx, nty, nb);
        if (zero)
            hipLaunchKernelGGL((k_rbgs_tile<T, D, true>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
        else
            hipLaunchKernelGGL((k_rbgs_tile<T, D, false>), dim3(nb), dim3(kThreads), 0, s, r, e_in, e_out, n, ntx, nty, co.a, co.invdiag);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_tile(int d, int n, const Coef<T>& co, const T* r, const T* e, T* rc, hipStream_t s) {
    const int nc = (n - 1) / 2;
    ISDC_DISPATCH_D(d, {
        int ntx, nty, nb;
        tile_counts<D>(nc, CTile<D>::X, CTile<D>::Y, CTile<D>::Z, ntx, nty, nb);
        hipLaunchKernelGGL((k_restrict_tile<T, D>), dim3(nb), dim3(kThreads), 0, s, r, e, rc, n, ntx, nty, co.a, co.diag);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_rbgs_tile(int d, int n, const Coef<T>& co, const T* r, const T* e_in, const T* ec,
                                    T* e_out, const double* g, double* u_out, int mode, hipStream_t s) {
    ISDC_DISPATCH_D(d, {
        int ntx, nty, nb;
        tile_counts<D>(n, Tile<D>::X, Tile<D>::Y, Tile<D>::Z, ntx, nty, nb);
        if (mode == 0)
            hipLaunchKernelGGL((k_prolong_rbgs_tile<T, D, 0>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
        else if (mode == 1)
            hipLaunchKernelGGL((k_prolong_rbgs_tile<T, D, 1>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
        else
            hipLaunchKernelGGL((k_prolong_rbgs_tile<T, D, 2>), dim3(nb), dim3(kThreads), 0, s, r, e_in, ec, e_out, n, ntx, nty, co.a, co.invdiag, g, u_out);
    });
    return hipGetLastError();
}

int tail_max_n(int d) {
    return d == 1 ? TailLayout<1>::nmax : (d == 2 ? TailLayout<2>::nmax : TailLayout<3>::nmax);
}

template <typename T>
hipError_t launch_tail(const MGConfig& cfg, int n, double c, double h, bool zero_guess, const T* rhs, T* e,
                       hipStream_t s) {
    if (n > tail_max_n(cfg.d)) return hipErrorInvalidValue;
    ISDC_DISPATCH_D(cfg.d, {
        hipLaunchKernelGGL((k_tail<T, D>), dim3(1), dim3(kTail), 0, s, rhs, e, n, c, h, cfg.smoother, cfg.nu_pre,
                           cfg.nu_post, cfg.omega, zero_guess ? 1 : 0);
    });
    return hipGetLastError();
}

#define ISDC_INST_T(T)                                                                                          \
    template hipError_t launch_rbgs_tile<T>(int, int, const Coef<T>&, bool, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_restrict_tile<T>(int, int, const Coef<T>&, const T*, const T*, T*, hipStream_t); \
    template hipError_t launch_prolong_rbgs_tile<T>(int, int, const Coef<T>&, const T*, const T*, const T*, T*,  \
                                                    const double*, double*, int, hipStream_t);                  \
    template hipError_t launch_tail<T>(const MGConfig&, int, double, double, bool, const T*, T*, hipStream_t);

ISDC_INST_T(float)
ISDC_INST_T(double)

}  // namespace isdc
