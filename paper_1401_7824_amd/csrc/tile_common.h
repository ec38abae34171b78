// Tiling helpers shared by the LDS-tiled kernels (device code).
//
// A launch covers the grid with tiles of Tile<D> points, one workgroup per
// tile.  Workgroups are renumbered so that each of the 8 XCDs (the hardware
// hands workgroup b to XCD b mod 8) gets a contiguous band of tiles, which
// keeps halo re-reads inside one XCD's L2.
#pragma once

#include <hip/hip_runtime.h>

namespace isdc {
namespace {

constexpr int kThreads = 256;

template <int D> struct Tile;
template <> struct Tile<1> { static constexpr int X = 1024, Y = 1, Z = 1; };
template <> struct Tile<2> { static constexpr int X = 64, Y = 16, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 32, Y = 8, Z = 4; };

// Shapes of the 1D and 3D multigrid tile kernels (2D levels use the row
// tiles of rows2d.h): shape 0 is Tile<D>, shapes 1 and 2 are smaller tiles
// (more workgroups, shorter per-workgroup latency chains, more halo per
// point).  A plan picks one per level (isdc_autotune).  Every extent is even,
// so a tile's coarse points start at its origin / 2.
constexpr int kShapes = 3;
template <int D, int S> struct TileS;
template <int D> struct TileS<D, 0> : Tile<D> {};
template <> struct TileS<1, 1> { static constexpr int X = 512, Y = 1, Z = 1; };
template <> struct TileS<1, 2> { static constexpr int X = 256, Y = 1, Z = 1; };
template <> struct TileS<3, 1> { static constexpr int X = 16, Y = 8, Z = 4; };
template <> struct TileS<3, 2> { static constexpr int X = 16, Y = 4, Z = 4; };

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

template <int D, int H, class TL>
using HaloBoxT = Box<D, TL::X + 2 * H, TL::Y + 2 * H, TL::Z + 2 * H>;
template <int D, int H>
using HaloBox = HaloBoxT<D, H, Tile<D>>;

// The element at byte offset off from p (a 32-bit per-thread offset from a
// uniform base: the saddr + voffset form of global loads and stores).
template <typename T>
__device__ __forceinline__ const T& at_byte(const T* p, unsigned off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
}
template <typename T>
__device__ __forceinline__ T& at_byte(T* p, unsigned off) {
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off);
}

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

// A box of a global array held in registers on its way to LDS: load() issues
// every load of this thread before any is waited on (a fully unrolled loop of
// compile-time length), store() writes them to LDS.  Outside the domain the
// box holds zeros (homogeneous Dirichlet ghosts).  Loading several boxes
// before storing any keeps all of a tile's global reads in flight at once.
template <typename T, int D, typename B>
struct Staged {
    static constexpr int kIter = (B::N + kThreads - 1) / kThreads;
    T v[kIter];
    __device__ __forceinline__ void load(const T* __restrict__ g, int n, int ox, int oy, int oz, bool zero) {
#pragma unroll
        for (int it = 0; it < kIter; ++it) {
            const int k = threadIdx.x + it * kThreads;
            int lx, ly, lz;
            B::split(k, lx, ly, lz);
            const int x = ox + lx, y = oy + ly, z = oz + lz;
            T val = T(0);
            if (!zero && k < B::N && inside<D>(x, y, z, n)) val = g[gidx<D>(x, y, z, n)];
            v[it] = val;
        }
    }
    __device__ __forceinline__ void store(T* s) const {
#pragma unroll
        for (int it = 0; it < kIter; ++it) {
            const int k = threadIdx.x + it * kThreads;
            if (k < B::N) s[k] = v[it];
        }
    }
};

template <typename T, int D, typename B>
__device__ __forceinline__ void stage(T* s, const T* __restrict__ g, int n, int ox, int oy, int oz, bool zero) {
    Staged<T, D, B> st;
    st.load(g, n, ox, oy, oz, zero);
    st.store(s);
}

// One pass over the points of box B in LDS: f(k, lx, ly, lz, v) returns the
// LDS index to write v to, or -1 for none.  All of a thread's values are
// computed before any is stored, so their LDS reads overlap; f must not read
// a location that another point of the same pass writes.
template <typename T, typename B, typename F>
__device__ __forceinline__ void lds_pass(T* s, F&& f) {
    constexpr int I = (B::N + kThreads - 1) / kThreads;
    T v[I];
    int at[I];
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int k = threadIdx.x + it * kThreads;
        int lx, ly, lz;
        B::split(k, lx, ly, lz);
        at[it] = k < B::N ? f(k, lx, ly, lz, v[it]) : -1;
    }
#pragma unroll
    for (int it = 0; it < I; ++it)
        if (at[it] >= 0) s[at[it]] = v[it];
}

// Visit the points of box B (fully unrolled; f(k, lx, ly, lz)).
template <typename B, typename F>
__device__ __forceinline__ void for_box(F&& f) {
    constexpr int I = (B::N + kThreads - 1) / kThreads;
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int k = threadIdx.x + it * kThreads;
        if (k >= B::N) break;
        int lx, ly, lz;
        B::split(k, lx, ly, lz);
        f(k, lx, ly, lz);
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
}  // namespace isdc
