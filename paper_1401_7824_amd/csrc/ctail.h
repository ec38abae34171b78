// Coarse tail of the compact stencil (device body): one V-cycle of
// B = I + w L_H - c A_H (the 9-point operator of eq. (5), rediscretised on
// every level) with weighted Jacobi smoothing, on a level of at most 63^2
// points (zero Dirichlet ghosts) or 32^2 points (periodic) and on every
// level below it, in one workgroup, with the level sizes known at compile
// time (one instantiation per top-level size).
//
// Dirichlet level of N = 2^k - 1 points per axis: the iterate has row stride
// N + 1, a zero ghost row above and below, and one more zero cell before and
// after, so all eight neighbours of a point are in the array (the zero at
// column N of row y is also the x = -1 neighbour of row y + 1) and read as
// zero outside the level: neighbour reads are immediate offsets with no
// boundary test.  Periodic level of N = 2^k points: stride N, neighbours wrap
// with a mask.  The right-hand side uses the iterate's strides without the
// leading ghost cells; each level has its own scratch array (residual for the
// restriction, the other half of the Jacobi ping-pong) with the iterate's
// layout.  Levels of at most 64 points run on the first wave alone.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "mg_device.h"

namespace isdc {
namespace {

template <bool PER, int N>
struct CL {
    static constexpr int S = PER ? N : N + 1;                        // row stride
    static constexpr int G = PER ? 0 : S + 1;                        // cells before point 0
    static constexpr int RN = N * S;                                 // right-hand side
    static constexpr int EN = PER ? N * N : (N + 2) * S + 2;         // iterate / scratch
    static constexpr int NP = N * N;
    static constexpr bool WAVE = NP <= 64;
    static constexpr int NT = WAVE ? 64 : kTail;
    static constexpr int Q = (NP + NT - 1) / NT;
    static constexpr int NC = PER ? N / 2 : (N - 1) / 2;
};
constexpr int kCTailMaxDirichlet = 63;

template <bool PER, int N>
constexpr int ct_etotal() {
    if constexpr (N == 1) return CL<PER, 1>::EN;
    else return CL<PER, N>::EN + ct_etotal<PER, CL<PER, N>::NC>();
}
template <bool PER, int N>
constexpr int ct_rtotal() {
    if constexpr (N == 1) return CL<PER, 1>::RN;
    else return CL<PER, N>::RN + ct_rtotal<PER, CL<PER, N>::NC>();
}

template <bool WAVE>
__device__ __forceinline__ void ct_sync() {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

// f(q, x, y) for this thread's points of the level.
template <bool PER, int N, typename F>
__device__ __forceinline__ void ct_plain(F&& f) {
    using Lv = CL<PER, N>;
#pragma unroll
    for (int q = 0; q < Lv::Q; ++q) {
        const int p = threadIdx.x + q * Lv::NT;
        if (p < Lv::NP) {
            const int y = p / N;
            f(q, p - y * N, y);
        }
    }
}

// B e at point (x, y): b0 e + bf (sum of the 4 edge neighbours) + bc (sum of
// the 4 corner neighbours), each sum in the order -x, +x, -y, +y (edges) and
// (-x,-y), (+x,-y), (-x,+y), (+x,+y) (corners).
template <bool PER, int N, typename T>
__device__ __forceinline__ T ct_apply(const T* e, int x, int y, T b0, T bf, T bc) {
    using Lv = CL<PER, N>;
    constexpr int S = Lv::S;
    if constexpr (PER) {
        constexpr int M = N - 1;
        const int xm = (x - 1) & M, xp = (x + 1) & M;
        const int ym = ((y - 1) & M) * S, y0 = y * S, yp = ((y + 1) & M) * S;
        const T edges = e[y0 + xm] + e[y0 + xp] + e[ym + x] + e[yp + x];
        const T corners = e[ym + xm] + e[ym + xp] + e[yp + xm] + e[yp + xp];
        return b0 * e[y0 + x] + bf * edges + bc * corners;
    } else {
        const int i = y * S + x;
        const T edges = e[i - 1] + e[i + 1] + e[i - S] + e[i + S];
        const T corners = e[i - S - 1] + e[i - S + 1] + e[i + S - 1] + e[i + S + 1];
        return b0 * e[i] + bf * edges + bc * corners;
    }
}

// nsteps weighted-Jacobi steps ping-ponging between e and the scratch t, the
// result copied back to e after an odd count.  zero: e is zero on entry, so
// the first step is (w r) / b0, which the full update gives for a zero iterate.
template <bool PER, int N, typename T>
__device__ __forceinline__ void ct_jacobi(T* e, const T* r, T* t, T b0, T bf, T bc, T w, int nsteps, bool zero) {
    using Lv = CL<PER, N>;
    constexpr int S = Lv::S;
    const T inv = T(1) / b0;
    T* src = e;
    T* dst = t;
    for (int k = 0; k < nsteps; ++k) {
        T v[Lv::Q];
        int at[Lv::Q];
#pragma unroll
        for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
        const bool z0 = k == 0 && zero;
        ct_plain<PER, N>([&](int q, int x, int y) {
            const int i = y * S + x;
            if (z0) v[q] = w * r[i] * inv;
            else v[q] = src[i] + w * (r[i] - ct_apply<PER, N>(src, x, y, b0, bf, bc)) * inv;
            at[q] = i;
        });
#pragma unroll
        for (int q = 0; q < Lv::Q; ++q)
            if (at[q] >= 0) dst[at[q]] = v[q];
        ct_sync<Lv::WAVE>();
        T* sw = src;
        src = dst;
        dst = sw;
    }
    if (src != e) {
        ct_plain<PER, N>([&](int, int x, int y) { e[y * S + x] = src[y * S + x]; });
        ct_sync<Lv::WAVE>();
    }
}

template <typename T, bool PER, int N, int L>
__device__ __forceinline__ void ct_level(T* eb, T* r, T* tb, const CTailCoefs& tc, int nu1, int nu2, T w, bool zero) {
    using Lv = CL<PER, N>;
    constexpr int S = Lv::S;
    T* e = eb + Lv::G;
    const T b0 = T(tc.b0[L]), bf = T(tc.bf[L]), bc = T(tc.bc[L]);
    if constexpr (N == 1) {
        // Dirichlet: every neighbour is a zero ghost; periodic: every
        // neighbour is the point itself and B = I
        if (threadIdx.x == 0) e[0] = PER ? r[0] : r[0] / b0;
        ct_sync<true>();
    } else {
        constexpr int NC = Lv::NC;
        using Lc = CL<PER, NC>;
        constexpr int SC = Lc::S;
        T* t = tb + Lv::G;
        T* ebc = eb + Lv::EN;
        T* ec = ebc + Lc::G;
        T* rc = r + Lv::RN;
        ct_jacobi<PER, N>(e, r, t, b0, bf, bc, w, nu1, zero);
        {
            T v[Lv::Q];
            int at[Lv::Q];
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
            ct_plain<PER, N>([&](int q, int x, int y) {
                v[q] = r[y * S + x] - ct_apply<PER, N>(e, x, y, b0, bf, bc);
                at[q] = y * S + x;
            });
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q)
                if (at[q] >= 0) t[at[q]] = v[q];
        }
        ct_sync<Lv::WAVE>();
        {
            // full weighting: Dirichlet coarse I on fine 2I+1, periodic on 2I
            const T wts[3] = {T(0.25), T(0.5), T(0.25)};
            ct_plain<PER, NC>([&](int, int X, int Y) {
                T acc = T(0);
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    if constexpr (PER) {
                        const int fy = ((2 * Y + oy - 1) & (N - 1)) * S;
                        const int fx0 = (2 * X - 1) & (N - 1);
                        acc += wts[oy] * (wts[0] * t[fy + fx0] + wts[1] * t[fy + 2 * X] + wts[2] * t[fy + 2 * X + 1]);
                    } else {
                        const int base = (2 * Y + oy) * S + 2 * X;
                        acc += wts[oy] * (wts[0] * t[base] + wts[1] * t[base + 1] + wts[2] * t[base + 2]);
                    }
                }
                rc[Y * SC + X] = acc;
                ec[Y * SC + X] = T(0);
            });
        }
        ct_sync<Lv::WAVE>();
        if constexpr (!Lv::WAVE && Lc::WAVE) {
            if (threadIdx.x < 64) ct_level<T, PER, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, nu1, nu2, w, true);
            __syncthreads();
        } else {
            ct_level<T, PER, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, nu1, nu2, w, true);
        }
        {
            // e += P e_c (linear interpolation per axis)
            T v[Lv::Q];
            int at[Lv::Q];
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q) at[q] = -1;
            ct_plain<PER, N>([&](int q, int x, int y) {
                T p;
                if constexpr (PER) {
                    // fine 2I on coarse I, fine 2I+1 the mean of I and I+1 (wrapping)
                    const int X0 = x >> 1, Y0 = y >> 1;
                    const int X1 = (x & 1) ? ((X0 + 1) & (NC - 1)) : X0;
                    const int Y1 = (y & 1) ? ((Y0 + 1) & (NC - 1)) : Y0;
                    const T wx = (x & 1) ? T(0.5) : T(1), wy = (y & 1) ? T(0.5) : T(1);
                    const T wx1 = (x & 1) ? T(0.5) : T(0), wy1 = (y & 1) ? T(0.5) : T(0);
                    p = wy * (wx * ec[Y0 * SC + X0] + wx1 * ec[Y0 * SC + X1]) +
                        wy1 * (wx * ec[Y1 * SC + X0] + wx1 * ec[Y1 * SC + X1]);
                } else {
                    // fine 2I+1 on coarse I, fine 2I the mean of I-1 and I (zero ghosts)
                    const T wx0 = (x & 1) ? T(1) : T(0.5), wx1 = (x & 1) ? T(0) : T(0.5);
                    const T wy0 = (y & 1) ? T(1) : T(0.5), wy1 = (y & 1) ? T(0) : T(0.5);
                    const int b = ((y - 1) >> 1) * SC + ((x - 1) >> 1);
                    p = wy0 * (wx0 * ec[b] + wx1 * ec[b + 1]) + wy1 * (wx0 * ec[b + SC] + wx1 * ec[b + SC + 1]);
                }
                v[q] = e[y * S + x] + p;
                at[q] = y * S + x;
            });
#pragma unroll
            for (int q = 0; q < Lv::Q; ++q)
                if (at[q] >= 0) e[at[q]] = v[q];
        }
        ct_sync<Lv::WAVE>();
        ct_jacobi<PER, N>(e, r, t, b0, bf, bc, w, nu2, false);
    }
}

template <typename T, bool PER, int NT>
__device__ __forceinline__ void ct_run(const T* __restrict__ rhs_g, T* __restrict__ e_g, T* E, T* R, T* TS,
                                       const CTailCoefs& tc, int nu1, int nu2, T w, int zero_guess) {
    using Lv = CL<PER, NT>;
    constexpr int S = Lv::S;
    constexpr int NE = ct_etotal<PER, NT>();
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
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) {
            const int y = p / NT, i = y * S + (p - y * NT);
            R[i] = vr[it];
            E[Lv::G + i] = ve[it];
        }
    }
    __syncthreads();
    if constexpr (Lv::WAVE) {
        if (threadIdx.x < 64) ct_level<T, PER, NT, 0>(E, R, TS, tc, nu1, nu2, w, zero_guess != 0);
        __syncthreads();
    } else {
        ct_level<T, PER, NT, 0>(E, R, TS, tc, nu1, nu2, w, zero_guess != 0);
    }
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) {
            const int y = p / NT;
            e_g[p] = E[Lv::G + y * S + (p - y * NT)];
        }
    }
}

// Entry: n_t = 2^k - 1 <= 63 (Dirichlet) or 2^k <= 32 (periodic); the
// launcher rejects other sizes.
template <typename T, bool PER>
__device__ __forceinline__ void ctail_body(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t,
                                           const CTailCoefs& tc, int nu1, int nu2, double omega, int zero_guess) {
    constexpr int NMAX = PER ? kCTailMaxPeriodic : kCTailMaxDirichlet;
    __shared__ T E[ct_etotal<PER, NMAX>()];
    __shared__ T R[ct_rtotal<PER, NMAX>()];
    __shared__ T TS[ct_etotal<PER, NMAX>()];
    const T w = T(omega);
    if constexpr (PER) {
        switch (n_t) {
            case 32: ct_run<T, true, 32>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 16: ct_run<T, true, 16>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 8: ct_run<T, true, 8>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 4: ct_run<T, true, 4>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 2: ct_run<T, true, 2>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            default: ct_run<T, true, 1>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
        }
    } else {
        switch (n_t) {
            case 63: ct_run<T, false, 63>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 31: ct_run<T, false, 31>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 15: ct_run<T, false, 15>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 7: ct_run<T, false, 7>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            case 3: ct_run<T, false, 3>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
            default: ct_run<T, false, 1>(rhs_g, e_g, E, R, TS, tc, nu1, nu2, w, zero_guess); break;
        }
    }
}

}  // namespace
}  // namespace isdc
