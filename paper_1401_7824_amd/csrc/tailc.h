// Coarse tail (device body): the V-cycle on a small level and on every level
// below it, in one workgroup, with the level sizes known at compile time (one
// instantiation per top-level size; at most 2047 points in 1D, 63^2 in 2D,
// 15^3 in 3D).
//
// A level of N points per axis stores its iterate with zero ghost cells:
// 1D  x + 1 in an array of N + 2;
// 2D  (y + 1) (N + 1) + x: row stride N + 1 and a ghost row above and below;
//     the zero at column N of row y is also the x = -1 neighbour of row y + 1;
// 3D  (z + 1) (N + 1)^2 + y (N + 1) + x: the same in every plane, where row N
//     of plane z (zero) is also the y = -1 row of plane z + 1, and a ghost
//     plane in front and behind.
// Every neighbour of a point is in the array and reads as zero outside the
// level, so the neighbour reads are immediate offsets with no boundary test.
// The right-hand side uses the same strides without the leading ghost row
// (plane); each level has its own scratch array (residual for the
// restriction, the other half of a Jacobi ping-pong) with the iterate's
// layout.  The arithmetic is that of the V-cycle of Sec. 3 as the tiled
// kernels compute it: neighbour sums in the order x, y, z; full weighting
// as a weighted sum of weighted rows; the prolongation e += P e_c is its own
// phase before the post-smoothing.
//
// Levels of at most 64 points run on the first wave alone with wave-level
// ordering instead of workgroup barriers.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "mg_device.h"

namespace isdc {
namespace {

// Level of N points per axis in D dimensions.
template <int D, int N>
struct LC {
    static constexpr int SY = D >= 2 ? N + 1 : 0;                // row stride
    static constexpr int SZ = D == 3 ? (N + 1) * (N + 1) : 0;    // plane stride
    static constexpr int G = D == 1 ? 1 : (D == 2 ? SY : SZ);    // ghost cells before point 0
    static constexpr int RN = D == 1 ? N : (D == 2 ? N * SY : N * SZ);  // right-hand side
    static constexpr int EN = RN + 2 * G;                        // iterate / scratch
    static constexpr int NP = D == 1 ? N : (D == 2 ? N * N : N * N * N);
    static constexpr int ROWS = NP / N;                          // rows along x
    static constexpr int HN = (N + 1) / 2;                       // colour slots per row
    static constexpr bool WAVE = NP <= 64;
    static constexpr int NT = WAVE ? 64 : kTail;                 // threads taking part
    static constexpr int Q = (NP + NT - 1) / NT;                 // plain slots per thread
    static constexpr int QC = (HN * ROWS + NT - 1) / NT;         // colour slots per thread
    // array index of point (x, y, z) relative to point 0
    __device__ static __forceinline__ int at(int x, int y, int z) { return z * SZ + y * SY + x; }
};
template <int D> constexpr int kTailMax = D == 1 ? 2047 : (D == 2 ? 63 : 15);

template <int D, int N>
constexpr int tc_etotal() {
    if constexpr (N == 1) return LC<D, 1>::EN;
    else return LC<D, N>::EN + tc_etotal<D, (N - 1) / 2>();
}
template <int D, int N>
constexpr int tc_rtotal() {
    if constexpr (N == 1) return LC<D, 1>::RN;
    else return LC<D, N>::RN + tc_rtotal<D, (N - 1) / 2>();
}

template <bool WAVE>
__device__ __forceinline__ void tc_sync() {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

// Sum of the 2D neighbours of index i, in the order x, y, z.
template <int D, int N, typename T>
__device__ __forceinline__ T tc_nb(const T* e, int i) {
    using Lv = LC<D, N>;
    T s = e[i - 1] + e[i + 1];
    if constexpr (D >= 2) s += e[i - Lv::SY] + e[i + Lv::SY];
    if constexpr (D == 3) s += e[i - Lv::SZ] + e[i + Lv::SZ];
    return s;
}

// f(q, x, y, z) for this thread's points of the level (q < Q).
template <int D, int N, typename F>
__device__ __forceinline__ void tc_plain(F&& f) {
    using Lv = LC<D, N>;
#pragma unroll
    for (int q = 0; q < Lv::Q; ++q) {
        const int p = threadIdx.x + q * Lv::NT;
        if (p < Lv::NP) {
            const int row = p / N;
            f(q, p - row * N, D >= 2 ? row % N : 0, D == 3 ? row / N : 0);
        }
    }
}

// One colour ((x + y + z) & 1 == colour) of a red-black step on the iterate e
// (point 0 of the level's array): the slots of a row hold every other x, so
// every slot of this thread holds a point of the colour.  ZERO: the iterate is
// zero, so the update is r * invdiag (the same value: a zero neighbour sum
// adds exactly nothing) and no neighbour is read.
template <int D, int N, bool ZERO = false, typename T>
__device__ __forceinline__ void tc_colour(T* e, const T* r, int colour, T a, T invdiag) {
    using Lv = LC<D, N>;
    constexpr int SL = Lv::HN * Lv::ROWS;
    T v[Lv::QC];
    int at[Lv::QC];
#pragma unroll
    for (int q = 0; q < Lv::QC; ++q) {
        const int s = threadIdx.x + q * Lv::NT;
        const int row = s / Lv::HN;
        const int y = D >= 2 ? row % N : 0, z = D == 3 ? row / N : 0;
        const int x = 2 * (s - row * Lv::HN) + ((y + z + colour) & 1);
        at[q] = -1;
        if (s < SL && x < N) {
            const int i = Lv::at(x, y, z);
            if (ZERO) v[q] = r[i] * invdiag;
            else v[q] = (r[i] + a * tc_nb<D, N>(e, i)) * invdiag;
            at[q] = i;
        }
    }
#pragma unroll
    for (int q = 0; q < Lv::QC; ++q)
        if (at[q] >= 0) e[at[q]] = v[q];
}

// nsteps smoothing steps (red-black in place; Jacobi ping-pongs between e and
// the scratch t and copies back after an odd count).  zero: e is zero on
// entry, so the first step reads no iterate (Jacobi: w (r invdiag), which is
// what the full update gives for a zero iterate).
template <int D, int N, typename T>
__device__ __forceinline__ void tc_smooth(T* e, const T* r, T* t, T a, T diag, T invdiag, T w, int smoother,
                                          int nsteps, bool zero) {
    using Lv = LC<D, N>;
    if (smoother == ISDC_SMOOTH_RBGS) {
        for (int k = 0; k < nsteps; ++k) {
            if (k == 0 && zero) tc_colour<D, N, true>(e, r, 0, a, invdiag);
            else tc_colour<D, N>(e, r, 0, a, invdiag);
            tc_sync<Lv::WAVE>();
            tc_colour<D, N>(e, r, 1, a, invdiag);
            tc_sync<Lv::WAVE>();
        }
        return;
    }
    T* src = e;
    T* dst = t;
    for (int k = 0; k < nsteps; ++k) {
        T v[Lv::Q];
        int at[Lv::Q];
#pragma unroll
        for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
        const bool z0 = k == 0 && zero;
        tc_plain<D, N>([&](int q, int x, int y, int z) {
            const int i = Lv::at(x, y, z);
            if (z0) {
                v[q] = w * (r[i] * invdiag);
            } else {
                const T c = src[i];
                v[q] = c + w * ((r[i] - (diag * c - a * tc_nb<D, N>(src, i))) * invdiag);
            }
            at[q] = i;
        });
#pragma unroll
        for (int q = 0; q < Lv::Q; ++q)
            if (at[q] >= 0) dst[at[q]] = v[q];
        tc_sync<Lv::WAVE>();
        T* sw = src;
        src = dst;
        dst = sw;
    }
    if (src != e) {
        tc_plain<D, N>([&](int, int x, int y, int z) { e[Lv::at(x, y, z)] = src[Lv::at(x, y, z)]; });
        tc_sync<Lv::WAVE>();
    }
}

// The V-cycle on level L (N points per axis) and below.  eb / tb: the level's
// iterate / scratch arrays from their first (ghost) cell; r: its right-hand
// side.  The next level's arrays follow each array directly.  zero: the
// iterate is zero on entry.
template <typename T, int D, int N, int L>
__device__ __forceinline__ void tc_level(T* eb, T* r, T* tb, const TailCoefs& tc, int smoother, int nu1, int nu2,
                                         T w, bool zero) {
    using Lv = LC<D, N>;
    T* e = eb + Lv::G;
    const T a = T(tc.a[L]), diag = T(tc.diag[L]), invdiag = T(tc.invdiag[L]);
    if constexpr (N == 1) {
        if (threadIdx.x == 0) e[0] = r[0] / diag;
        tc_sync<true>();
    } else {
        constexpr int NC = (N - 1) / 2;
        using Lc = LC<D, NC>;
        T* t = tb + Lv::G;
        T* ebc = eb + Lv::EN;
        T* ec = ebc + Lc::G;
        T* rc = r + Lv::RN;
        tc_smooth<D, N>(e, r, t, a, diag, invdiag, w, smoother, nu1, zero);
        {
            // residual into the scratch
            T v[Lv::Q];
            int at[Lv::Q];
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
            tc_plain<D, N>([&](int q, int x, int y, int z) {
                const int i = Lv::at(x, y, z);
                v[q] = r[i] - (diag * e[i] - a * tc_nb<D, N>(e, i));
                at[q] = i;
            });
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q)
                if (at[q] >= 0) t[at[q]] = v[q];
        }
        tc_sync<Lv::WAVE>();
        {
            // full weighting onto the coarse level (fine 2I, 2I+1, 2I+2 per
            // axis), whose iterate starts at zero
            const T wt[3] = {T(0.25), T(0.5), T(0.25)};
            tc_plain<D, NC>([&](int, int X, int Y, int Z) {
                const int b = Lv::at(2 * X, 2 * Y, 2 * Z);
                T acc = T(0);
#pragma unroll
                for (int oz = 0; oz < (D == 3 ? 3 : 1); ++oz)
#pragma unroll
                    for (int oy = 0; oy < (D >= 2 ? 3 : 1); ++oy) {
                        const int c = b + oz * Lv::SZ + oy * Lv::SY;
                        const T row = wt[0] * t[c] + wt[1] * t[c + 1] + wt[2] * t[c + 2];
                        acc += (D >= 2 ? wt[oy] : T(1)) * (D == 3 ? wt[oz] : T(1)) * row;
                    }
                const int I = Lc::at(X, Y, Z);
                rc[I] = acc;
                ec[I] = T(0);
            });
        }
        tc_sync<Lv::WAVE>();
        if constexpr (!Lv::WAVE && Lc::WAVE) {
            if (threadIdx.x < 64) tc_level<T, D, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, smoother, nu1, nu2, w, true);
            __syncthreads();
        } else {
            tc_level<T, D, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, smoother, nu1, nu2, w, true);
        }
        {
            // e += P e_c: per axis an odd index takes coarse point (i-1)/2, an
            // even one the mean of i/2-1 and i/2 (ghosts are zero, and a zero
            // weight times a stored value adds exactly nothing)
            T v[Lv::Q];
            int at[Lv::Q];
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
            tc_plain<D, N>([&](int q, int x, int y, int z) {
                const T wx0 = (x & 1) ? T(1) : T(0.5), wx1 = (x & 1) ? T(0) : T(0.5);
                const int b = Lc::at((x - 1) >> 1, D >= 2 ? (y - 1) >> 1 : 0, D == 3 ? (z - 1) >> 1 : 0);
                auto rowv = [&](int o) { return wx0 * ec[o] + wx1 * ec[o + 1]; };
                T p;
                if constexpr (D == 1) {
                    p = rowv(b);
                } else {
                    const T wy0 = (y & 1) ? T(1) : T(0.5), wy1 = (y & 1) ? T(0) : T(0.5);
                    auto plane = [&](int o) { return wy0 * rowv(o) + wy1 * rowv(o + Lc::SY); };
                    if constexpr (D == 2) {
                        p = plane(b);
                    } else {
                        const T wz0 = (z & 1) ? T(1) : T(0.5), wz1 = (z & 1) ? T(0) : T(0.5);
                        p = wz0 * plane(b) + wz1 * plane(b + Lc::SZ);
                    }
                }
                const int i = Lv::at(x, y, z);
                v[q] = e[i] + p;
                at[q] = i;
            });
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q)
                if (at[q] >= 0) e[at[q]] = v[q];
        }
        tc_sync<Lv::WAVE>();
        tc_smooth<D, N>(e, r, t, a, diag, invdiag, w, smoother, nu2, false);
    }
}

// The whole tail from a top level of NT points per axis: stage the level's
// right-hand side (and iterate) from global memory, run the V-cycle, write the
// iterate back.  E, R, TS: LDS arrays of tc_etotal / tc_rtotal / tc_etotal
// entries for kTailMax<D>.
template <typename T, int D, int NT>
__device__ __forceinline__ void tc_run(const T* __restrict__ rhs_g, T* __restrict__ e_g, T* E, T* R, T* TS,
                                       const TailCoefs& tc, int smoother, int nu1, int nu2, T w, int zero_guess) {
    using Lv = LC<D, NT>;
    constexpr int NE = tc_etotal<D, NT>();
    // zero every iterate and scratch array (their ghosts stay zero)
    for (int k = threadIdx.x; k < NE; k += kTail) {
        E[k] = T(0);
        TS[k] = T(0);
    }
    __syncthreads();
    constexpr int I = (Lv::NP + kTail - 1) / kTail;
    T vr[I], ve[I];
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        vr[it] = p < Lv::NP ? rhs_g[p] : T(0);
        ve[it] = (p < Lv::NP && !zero_guess) ? e_g[p] : T(0);
    }
    auto index = [](int p) {
        const int row = p / NT;
        return Lv::at(p - row * NT, D >= 2 ? row % NT : 0, D == 3 ? row / NT : 0);
    };
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) {
            const int i = index(p);
            R[i] = vr[it];
            E[Lv::G + i] = ve[it];
        }
    }
    __syncthreads();
    if constexpr (Lv::WAVE) {
        if (threadIdx.x < 64) tc_level<T, D, NT, 0>(E, R, TS, tc, smoother, nu1, nu2, w, zero_guess != 0);
        __syncthreads();
    } else {
        tc_level<T, D, NT, 0>(E, R, TS, tc, smoother, nu1, nu2, w, zero_guess != 0);
    }
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) e_g[p] = E[Lv::G + index(p)];
    }
}

// Tail entry: n_t = 2^k - 1 up to kTailMax<D> (the launcher rejects others).
template <typename T, int D>
__device__ __forceinline__ void tailc_body(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t,
                                           const TailCoefs& tc, int smoother, int nu1, int nu2, double omega,
                                           int zero_guess) {
    __shared__ T E[tc_etotal<D, kTailMax<D>>()];
    __shared__ T R[tc_rtotal<D, kTailMax<D>>()];
    __shared__ T TS[tc_etotal<D, kTailMax<D>>()];
    const T w = T(omega);
#define ISDC_TC_CASE(NV)                                                                                   \
    case NV:                                                                                               \
        if constexpr (NV <= kTailMax<D>) tc_run<T, D, NV>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); \
        break;
    switch (n_t) {
        ISDC_TC_CASE(2047)
        ISDC_TC_CASE(1023)
        ISDC_TC_CASE(511)
        ISDC_TC_CASE(255)
        ISDC_TC_CASE(127)
        ISDC_TC_CASE(63)
        ISDC_TC_CASE(31)
        ISDC_TC_CASE(15)
        ISDC_TC_CASE(7)
        ISDC_TC_CASE(3)
        default: tc_run<T, D, 1>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
    }
#undef ISDC_TC_CASE
}

}  // namespace
}  // namespace isdc
