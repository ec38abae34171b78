// Coarse tail for 2D levels (device body): the V-cycle on a level of at most
// 63^2 points and on every level below it, in one workgroup, with the level
// sizes known at compile time (one instantiation per top-level size).
//
// A level of N points per axis stores its iterate with row stride N + 1 and
// a zero ghost row above and below: the zero at column N of row y is also the
// x = -1 neighbour of row y + 1, so every neighbour of a point is in the
// array, ghosts read as zero, and the four neighbour reads are immediate
// offsets with no boundary test.  The right-hand side uses the same stride
// without ghost rows; each level has its own scratch array (residual for the
// restriction, the other half of a Jacobi ping-pong) with the iterate's
// layout.  The arithmetic is that of tail_body in mg_device.h, term for term;
// the prolongation is a separate phase e += P e_c before the post-smoothing.
//
// Levels of at most 64 points run on the first wave alone with wave-level
// ordering instead of workgroup barriers.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"
#include "mg_device.h"

namespace isdc {
namespace {

template <int N>
struct L2 {
    static constexpr int S = N + 1;         // row stride
    static constexpr int EN = (N + 2) * S;  // iterate / scratch, with ghost rows
    static constexpr int RN = N * S;        // right-hand side
    static constexpr int NP = N * N;
    static constexpr int HN = (N + 1) / 2;  // colour slots per row
    static constexpr bool WAVE = NP <= 64;
    static constexpr int NT = WAVE ? 64 : kTail;  // threads taking part
};

template <int N>
constexpr int t2_etotal() {
    if constexpr (N == 1) return L2<1>::EN;
    else return L2<N>::EN + t2_etotal<(N - 1) / 2>();
}
template <int N>
constexpr int t2_rtotal() {
    if constexpr (N == 1) return L2<1>::RN;
    else return L2<N>::RN + t2_rtotal<(N - 1) / 2>();
}
constexpr int kT2Max = 63;  // largest top level (= TailLayout<2>::nmax)

template <bool WAVE>
__device__ __forceinline__ void t2_sync() {
    if constexpr (WAVE) wave_sync();
    else __syncthreads();
}

// f(q, x, y) for this thread's points of an N^2 level (q < Q = slots per thread).
template <int N, typename F>
__device__ __forceinline__ void t2_plain(F&& f) {
    using Lv = L2<N>;
    constexpr int Q = (Lv::NP + Lv::NT - 1) / Lv::NT;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int p = threadIdx.x + q * Lv::NT;
        if (p < Lv::NP) {
            const int y = p / N;
            f(q, p - y * N, y);
        }
    }
}

// One colour of a red-black step on the iterate e (row 0 of the level's
// array): every slot of this thread holds a point of the colour.  ZERO: the
// iterate is zero, so the update is r * invdiag (the same value: a zero
// neighbour sum adds exactly nothing) and no neighbour is read.
template <int N, bool ZERO = false, typename T>
__device__ __forceinline__ void t2_colour(T* e, const T* r, int colour, T a, T invdiag) {
    using Lv = L2<N>;
    constexpr int S = Lv::S, SL = N * Lv::HN;
    constexpr int Q = (SL + Lv::NT - 1) / Lv::NT;
    T v[Q];
    int at[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int s = threadIdx.x + q * Lv::NT;
        const int y = s / Lv::HN;
        const int x = 2 * (s - y * Lv::HN) + ((y + colour) & 1);
        at[q] = -1;
        if (s < SL && x < N) {
            const int i = y * S + x;
            if (ZERO) v[q] = r[i] * invdiag;
            else v[q] = (r[i] + a * (e[i - 1] + e[i + 1] + e[i - S] + e[i + S])) * invdiag;
            at[q] = i;
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (at[q] >= 0) e[at[q]] = v[q];
}

// nsteps smoothing steps (red-black in place; Jacobi ping-pongs between e and
// the scratch t and copies back after an odd count).  zero: e is zero on
// entry, so the first step reads no iterate (Jacobi: w (r invdiag), which is
// what the full update gives for a zero iterate).
template <int N, typename T>
__device__ __forceinline__ void t2_smooth(T* e, const T* r, T* t, T a, T diag, T invdiag, T w, int smoother,
                                          int nsteps, bool zero) {
    using Lv = L2<N>;
    constexpr int S = Lv::S;
    constexpr int Q = (Lv::NP + Lv::NT - 1) / Lv::NT;
    if (smoother == ISDC_SMOOTH_RBGS) {
        for (int k = 0; k < nsteps; ++k) {
            if (k == 0 && zero) t2_colour<N, true>(e, r, 0, a, invdiag);
            else t2_colour<N>(e, r, 0, a, invdiag);
            t2_sync<Lv::WAVE>();
            t2_colour<N>(e, r, 1, a, invdiag);
            t2_sync<Lv::WAVE>();
        }
        return;
    }
    T* src = e;
    T* dst = t;
    for (int k = 0; k < nsteps; ++k) {
        T v[Q];
        int at[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) at[q] = -1;
        const bool z = k == 0 && zero;
        t2_plain<N>([&](int q, int x, int y) {
            const int i = y * S + x;
            if (z) {
                v[q] = w * (r[i] * invdiag);
            } else {
                const T c = src[i];
                v[q] = c + w * ((r[i] - (diag * c - a * (src[i - 1] + src[i + 1] + src[i - S] + src[i + S]))) *
                                invdiag);
            }
            at[q] = i;
        });
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (at[q] >= 0) dst[at[q]] = v[q];
        t2_sync<Lv::WAVE>();
        T* sw = src;
        src = dst;
        dst = sw;
    }
    if (src != e) {
        t2_plain<N>([&](int, int x, int y) { e[y * S + x] = src[y * S + x]; });
        t2_sync<Lv::WAVE>();
    }
}

// The V-cycle on level L (N points per axis) and below.  eb / tb: the level's
// iterate / scratch arrays including the ghost row above; r: its right-hand
// side.  The next level's arrays follow each array directly.
template <typename T, int N, int L>
__device__ __forceinline__ void t2_level(T* eb, T* r, T* tb, const TailCoefs& tc, int smoother, int nu1, int nu2,
                                         T w, bool zero) {
    using Lv = L2<N>;
    constexpr int S = Lv::S;
    T* e = eb + S;
    const T a = T(tc.a[L]), diag = T(tc.diag[L]), invdiag = T(tc.invdiag[L]);
    if constexpr (N == 1) {
        if (threadIdx.x == 0) e[0] = r[0] / diag;
        t2_sync<true>();
    } else {
        constexpr int NC = (N - 1) / 2;
        using Lc = L2<NC>;
        constexpr int SC = Lc::S;
        T* t = tb + S;
        T* ebc = eb + Lv::EN;
        T* ec = ebc + SC;
        T* rc = r + Lv::RN;
        t2_smooth<N>(e, r, t, a, diag, invdiag, w, smoother, nu1, zero);
        {
            // residual into the scratch
            constexpr int Q = (Lv::NP + Lv::NT - 1) / Lv::NT;
            T v[Q];
            int at[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) at[q] = -1;
            t2_plain<N>([&](int q, int x, int y) {
                const int i = y * S + x;
                v[q] = r[i] - (diag * e[i] - a * (e[i - 1] + e[i + 1] + e[i - S] + e[i + S]));
                at[q] = i;
            });
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (at[q] >= 0) t[at[q]] = v[q];
        }
        t2_sync<Lv::WAVE>();
        {
            // full weighting onto the coarse level, whose iterate starts at zero
            const T w0 = T(0.25), w1 = T(0.5);
            t2_plain<NC>([&](int, int X, int Y) {
                const int b = 2 * Y * S + 2 * X;
                const T q0 = w0 * t[b] + w1 * t[b + 1] + w0 * t[b + 2];
                const T q1 = w0 * t[b + S] + w1 * t[b + S + 1] + w0 * t[b + S + 2];
                const T q2 = w0 * t[b + 2 * S] + w1 * t[b + 2 * S + 1] + w0 * t[b + 2 * S + 2];
                T acc = T(0);
                acc += w0 * q0;
                acc += w1 * q1;
                acc += w0 * q2;
                rc[Y * SC + X] = acc;
                ec[Y * SC + X] = T(0);
            });
        }
        t2_sync<Lv::WAVE>();
        if constexpr (!Lv::WAVE && Lc::WAVE) {
            if (threadIdx.x < 64) t2_level<T, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, smoother, nu1, nu2, w, true);
            __syncthreads();
        } else {
            t2_level<T, NC, L + 1>(ebc, rc, tb + Lv::EN, tc, smoother, nu1, nu2, w, true);
        }
        {
            // e += P e_c: per axis an odd index takes coarse point (i-1)/2, an
            // even one the mean of i/2-1 and i/2 (ghosts are zero)
            constexpr int Q = (Lv::NP + Lv::NT - 1) / Lv::NT;
            T v[Q];
            int at[Q];
#pragma unroll
            for (int q = 0; q < Q; ++q) at[q] = -1;
            t2_plain<N>([&](int q, int x, int y) {
                const int xa = (x - 1) >> 1, ya = (y - 1) >> 1;
                const T wx0 = (x & 1) ? T(1) : T(0.5), wx1 = (x & 1) ? T(0) : T(0.5);
                const T wy0 = (y & 1) ? T(1) : T(0.5), wy1 = (y & 1) ? T(0) : T(0.5);
                const int b = ya * SC + xa;
                const T p0 = wx0 * ec[b] + wx1 * ec[b + 1];
                const T p1 = wx0 * ec[b + SC] + wx1 * ec[b + SC + 1];
                const int i = y * S + x;
                v[q] = e[i] + (wy0 * p0 + wy1 * p1);
                at[q] = i;
            });
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (at[q] >= 0) e[at[q]] = v[q];
        }
        t2_sync<Lv::WAVE>();
        t2_smooth<N>(e, r, t, a, diag, invdiag, w, smoother, nu2, false);
    }
}

// The whole tail from a top level of NT points per axis: stage the level's
// right-hand side (and iterate) from global memory, run the V-cycle, write the
// iterate back.  E, R, TS: LDS arrays of t2_etotal / t2_rtotal / t2_etotal
// entries for kT2Max.
template <typename T, int NT>
__device__ __forceinline__ void t2_run(const T* __restrict__ rhs_g, T* __restrict__ e_g, T* E, T* R, T* TS,
                                       const TailCoefs& tc, int smoother, int nu1, int nu2, T w, int zero_guess) {
    using Lv = L2<NT>;
    constexpr int S = Lv::S;
    constexpr int NE = t2_etotal<NT>();
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
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) {
            const int y = p / NT, x = p - y * NT;
            R[y * S + x] = vr[it];
            E[(y + 1) * S + x] = ve[it];
        }
    }
    __syncthreads();
    if constexpr (Lv::WAVE) {
        if (threadIdx.x < 64) t2_level<T, NT, 0>(E, R, TS, tc, smoother, nu1, nu2, w, zero_guess != 0);
        __syncthreads();
    } else {
        t2_level<T, NT, 0>(E, R, TS, tc, smoother, nu1, nu2, w, zero_guess != 0);
    }
#pragma unroll
    for (int it = 0; it < I; ++it) {
        const int p = threadIdx.x + it * kTail;
        if (p < Lv::NP) {
            const int y = p / NT, x = p - y * NT;
            e_g[p] = E[(y + 1) * S + x];
        }
    }
}

// 2D tail entry: n_t in {1, 3, 7, 15, 31, 63} (others are rejected by the launcher).
template <typename T>
__device__ __forceinline__ void tail2_body(const T* __restrict__ rhs_g, T* __restrict__ e_g, int n_t,
                                           const TailCoefs& tc, int smoother, int nu1, int nu2, double omega,
                                           int zero_guess) {
    __shared__ T E[t2_etotal<kT2Max>()];
    __shared__ T R[t2_rtotal<kT2Max>()];
    __shared__ T TS[t2_etotal<kT2Max>()];
    const T w = T(omega);
    switch (n_t) {
        case 63: t2_run<T, 63>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
        case 31: t2_run<T, 31>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
        case 15: t2_run<T, 15>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
        case 7: t2_run<T, 7>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
        case 3: t2_run<T, 3>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
        default: t2_run<T, 1>(rhs_g, e_g, E, R, TS, tc, smoother, nu1, nu2, w, zero_guess); break;
    }
}

}  // namespace
}  // namespace isdc
