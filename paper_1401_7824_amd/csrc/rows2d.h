// Row-mapped 2D tiles: the red-black step, the red-black step fused with the
// residual's full-weighting restriction, and the prolongation fused with a
// red-black step, for 2D levels (device bodies; same arithmetic as the
// generic tile bodies of mg_device.h).
//
// Every LDS array of a tile has one layout: LPR columns x0-3 .. x0+LPR-4 by
// NR rows y0-3 .., row-major with stride LPR, for a tile of TX = LPR - 8 by
// TY points at (x0, y0) (the widest region a kernel touches is the tile plus
// a halo of 3, TX + 7 columns).  A thread keeps one column in a plain pass
// (t % LPR) and one colour parity in a colour pass, so the LDS address of
// each of its points is a per-thread constant plus a compile-time row offset
// and the four neighbours are immediate offsets; global addresses are a
// per-thread 32-bit byte offset plus a uniform row step.  The domain test
// folds into uniform bounds on the LDS column and row.
//
// Plain pass: thread t takes column t % LPR and rows t / LPR + i * RP
// (RP = 256 / LPR), i.e. LDS index t + 256 i.
// Colour pass: a row holds LPR/2 points of each colour, one every other
// column, so thread t takes colour lane t % (LPR/2) of rows t / (LPR/2) +
// i * RC (RC = 512 / LPR, even): its column parity is fixed per colour, and
// every lane of a wave has a point of the colour.
#pragma once

#include <hip/hip_runtime.h>

#include "tile_common.h"

namespace isdc {
namespace {

template <int LPR_, int TY_>
struct RowT {
    static constexpr int LPR = LPR_, TY = TY_;
    static constexpr int TX = LPR - 8;
    static constexpr int ROWS = TY + 7;  // y0-3 .. y0+TY+3
    static constexpr int RP = kThreads / LPR;
    static constexpr int IP = (ROWS + RP - 1) / RP;  // plain steps over the array
    static constexpr int NR = IP * RP;
    static constexpr int N = NR * LPR;  // = 256 IP
    static constexpr int H = LPR / 2;
    static constexpr int RC = kThreads / H;  // rows per colour step
    static constexpr int IC = (ROWS + RC - 1) / RC;
    static constexpr int CROWS = TY / 2 + 4;  // coarse rows staged by the prolongation
    static constexpr int ICP = (CROWS + RC - 1) / RC;
    static_assert(TX % 2 == 0 && TY % 2 == 0 && RC % 2 == 0, "even tiles and colour steps");
};
// the three row shapes of a 2D level
template <int S> struct RowShape;
template <> struct RowShape<0> { using RT = RowT<64, 16>; };
template <> struct RowShape<1> { using RT = RowT<64, 8>; };
template <> struct RowShape<2> { using RT = RowT<32, 8>; };

// A region of the layout in LDS coordinates (inclusive), clipped to the
// domain 0 <= x, y < n.
struct Region {
    int clo, chi, rlo, rhi;
};
__device__ __forceinline__ Region region(int h, int xr, int yr, int x0, int y0, int n, int TX, int TY) {
    // columns 3-h .. TX+2+h+xr, rows 3-h .. TY+2+h+yr (xr, yr: one extra
    // column / row on the high side, for the residual region)
    Region g;
    g.clo = max(3 - h, 3 - x0);
    g.chi = min(TX + 2 + h + xr, n + 2 - x0);
    g.rlo = max(3 - h, 3 - y0);
    g.rhi = min(TY + 2 + h + yr, n + 2 - y0);
    return g;
}

// Plain-pass loads of g over region gr into v (zero elsewhere).
template <class RT, typename T>
__device__ __forceinline__ void rows_load(T (&v)[RT::IP], const T* __restrict__ g, int n, int x0, int y0,
                                          const Region& gr) {
    const int c = threadIdx.x % RT::LPR, j = threadIdx.x / RT::LPR;
    const bool cok = c >= gr.clo && c <= gr.chi;
    const unsigned rowb = (unsigned)n * sizeof(T);
    const unsigned off0 = (unsigned)(y0 - 3 + j) * rowb + (unsigned)(x0 - 3 + c) * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < RT::IP; ++i) {
        const int row = j + i * RT::RP;
        T x = T(0);
        if (cok && row >= gr.rlo && row <= gr.rhi) x = at_byte(g, off0 + (unsigned)(i * RT::RP) * rowb);
        v[i] = x;
    }
}

template <class RT, typename T>
__device__ __forceinline__ void rows_store_lds(T* s, const T (&v)[RT::IP]) {
#pragma unroll
    for (int i = 0; i < RT::IP; ++i) s[threadIdx.x + i * kThreads] = v[i];
}

// Plain pass over region gr: f(k, i) for this thread's points (k = LDS index,
// i = step, for per-step registers).
template <class RT, typename F>
__device__ __forceinline__ void rows_plain(const Region& gr, F&& f) {
    const int c = threadIdx.x % RT::LPR, j = threadIdx.x / RT::LPR;
    if (c < gr.clo || c > gr.chi) return;
#pragma unroll
    for (int i = 0; i < RT::IP; ++i) {
        const int row = j + i * RT::RP;
        if (row >= gr.rlo && row <= gr.rhi) f(threadIdx.x + i * kThreads, i);
    }
}

// One colour of a red-black step over region gr, in place in se:
// v = (sr + a * (sum of the 4 neighbours)) * invdiag.  colour 0 = red
// ((x + y) even), 1 = black.  A colour reads only the other colour, so all
// of a thread's values are computed before any is stored.
template <class RT, typename T>
__device__ __forceinline__ void rows_colour(T* se, const T* sr, int colour, int x0, int y0, const Region& gr, T a,
                                            T invdiag) {
    constexpr int L = RT::LPR;
    const int cl = threadIdx.x % RT::H, rr = threadIdx.x / RT::H;
    // (x + y) = x0 + y0 - 6 + c + row has the colour's parity
    const int c = 2 * cl + ((x0 + y0 + rr + colour) & 1);
    if (c < gr.clo || c > gr.chi) return;
    const int base = rr * L + c;
    T v[RT::IC];
    bool w[RT::IC];
#pragma unroll
    for (int i = 0; i < RT::IC; ++i) {
        const int row = rr + i * RT::RC;
        const int k = base + i * RT::RC * L;
        w[i] = row >= gr.rlo && row <= gr.rhi;
        if (w[i]) v[i] = (sr[k] + a * (se[k - 1] + se[k + 1] + se[k - L] + se[k + L])) * invdiag;
    }
#pragma unroll
    for (int i = 0; i < RT::IC; ++i)
        if (w[i]) se[base + i * RT::RC * L] = v[i];
}

// Plain-pass stores of LDS values (through f(k, i) -> value) to global over gr.
template <class RT, typename TO, typename F>
__device__ __forceinline__ void rows_store(TO* __restrict__ out, int n, int x0, int y0, const Region& gr, F&& f) {
    const int c = threadIdx.x % RT::LPR, j = threadIdx.x / RT::LPR;
    if (c < gr.clo || c > gr.chi) return;
    const unsigned rowb = (unsigned)n * sizeof(TO);
    const unsigned off0 = (unsigned)(y0 - 3 + j) * rowb + (unsigned)(x0 - 3 + c) * (unsigned)sizeof(TO);
#pragma unroll
    for (int i = 0; i < RT::IP; ++i) {
        const int row = j + i * RT::RP;
        if (row >= gr.rlo && row <= gr.rhi)
            at_byte(out, off0 + (unsigned)(i * RT::RP) * rowb) = f(threadIdx.x + i * kThreads, i);
    }
}

// One red-black step from e_in to e_out (red on the tile plus a halo of 1,
// black on the tile).  ZERO: e_in is zero and not read.
template <typename T, bool ZERO, class RT>
__device__ __forceinline__ void rows_rbgs_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                               T* __restrict__ e_out, int n, int x0, int y0, T a, T invdiag) {
    __shared__ T se[RT::N];
    __shared__ T sr[RT::N];
    const Region R2 = region(2, 0, 0, x0, y0, n, RT::TX, RT::TY);
    const Region R1 = region(1, 0, 0, x0, y0, n, RT::TX, RT::TY);
    const Region T0 = region(0, 0, 0, x0, y0, n, RT::TX, RT::TY);
    {
        T ve[RT::IP], vr[RT::IP];
        if (ZERO) {
#pragma unroll
            for (int i = 0; i < RT::IP; ++i) ve[i] = T(0);
        } else {
            rows_load<RT>(ve, e_in, n, x0, y0, R2);
        }
        rows_load<RT>(vr, r, n, x0, y0, R1);
        rows_store_lds<RT>(se, ve);
        rows_store_lds<RT>(sr, vr);
    }
    __syncthreads();
    rows_colour<RT>(se, sr, 0, x0, y0, R1, a, invdiag);
    __syncthreads();
    rows_colour<RT>(se, sr, 1, x0, y0, T0, a, invdiag);
    __syncthreads();
    rows_store<RT>(e_out, n, x0, y0, T0, [&](int k, int) { return se[k]; });
}

// One red-black step from e_in to e_out fused with rc = full weighting of
// (r - A e_out): the new iterate is computed on the tile plus a halo of 1
// (red on a halo of 2), so the residual is known on every fine point under
// the tile's coarse points.  In two parts: rr_load fills registers, rr_run
// stores them to LDS and does the rest.
template <typename T, class RT>
struct RRStage {
    T ve[RT::IP], vr[RT::IP];
};

template <typename T, bool ZERO, class RT>
__device__ __forceinline__ void rr_load(RRStage<T, RT>& st, const T* __restrict__ r, const T* __restrict__ e_in,
                                        int n, int x0, int y0) {
    // the residual is needed on x0 .. x0+TX (one past the tile), so every
    // region below it reaches one point further on the high side
    if (ZERO) {
#pragma unroll
        for (int i = 0; i < RT::IP; ++i) st.ve[i] = T(0);
    } else {
        rows_load<RT>(st.ve, e_in, n, x0, y0, region(3, 1, 1, x0, y0, n, RT::TX, RT::TY));
    }
    rows_load<RT>(st.vr, r, n, x0, y0, region(2, 1, 1, x0, y0, n, RT::TX, RT::TY));
}

template <typename T, class RT>
__device__ __forceinline__ void rr_run(const RRStage<T, RT>& st, T* se, T* sr, T* __restrict__ e_out,
                                       T* __restrict__ rc, int n, int x0, int y0, T a, T diag, T invdiag) {
    constexpr int L = RT::LPR;
    const Region R2 = region(2, 1, 1, x0, y0, n, RT::TX, RT::TY);
    const Region R1 = region(1, 1, 1, x0, y0, n, RT::TX, RT::TY);
    const Region RS = region(0, 1, 1, x0, y0, n, RT::TX, RT::TY);  // x0 .. x0+TX, y0 .. y0+TY
    const Region T0 = region(0, 0, 0, x0, y0, n, RT::TX, RT::TY);
    rows_store_lds<RT>(se, st.ve);
    rows_store_lds<RT>(sr, st.vr);
    __syncthreads();
    rows_colour<RT>(se, sr, 0, x0, y0, R2, a, invdiag);
    __syncthreads();
    rows_colour<RT>(se, sr, 1, x0, y0, R1, a, invdiag);
    __syncthreads();
    rows_store<RT>(e_out, n, x0, y0, T0, [&](int k, int) { return se[k]; });
    {
        // residual in place of the rhs (reads only se and its own sr)
        T v[RT::IP];
        bool w[RT::IP];
#pragma unroll
        for (int i = 0; i < RT::IP; ++i) w[i] = false;
        rows_plain<RT>(RS, [&](int k, int i) {
            v[i] = sr[k] - (diag * se[k] - a * (se[k - 1] + se[k + 1] + se[k - L] + se[k + L]));
            w[i] = true;
        });
#pragma unroll
        for (int i = 0; i < RT::IP; ++i)
            if (w[i]) sr[threadIdx.x + i * kThreads] = v[i];
    }
    __syncthreads();
    // full weighting: coarse point (X, Y) = (x0/2 + cx, y0/2 + cy) from the
    // fine points 2cx + {0,1,2}, 2cy + {0,1,2} of the tile (LDS column / row 3 + ...)
    const int nc = (n - 1) / 2;
    const int cx = threadIdx.x % RT::H, cy0 = threadIdx.x / RT::H;
    const int X = x0 / 2 + cx;
    if (cx >= RT::TX / 2 || X >= nc) return;
    const T w0 = T(0.25), w1 = T(0.5);
#pragma unroll
    for (int i = 0; i < (RT::TY / 2 + RT::RC - 1) / RT::RC; ++i) {
        const int cy = cy0 + i * RT::RC;
        const int Y = y0 / 2 + cy;
        if (cy >= RT::TY / 2 || Y >= nc) continue;
        const int b = (3 + 2 * cy) * L + 3 + 2 * cx;
        const T r0 = w0 * sr[b] + w1 * sr[b + 1] + w0 * sr[b + 2];
        const T r1 = w0 * sr[b + L] + w1 * sr[b + L + 1] + w0 * sr[b + L + 2];
        const T r2 = w0 * sr[b + 2 * L] + w1 * sr[b + 2 * L + 1] + w0 * sr[b + 2 * L + 2];
        T acc = T(0);
        acc += w0 * r0;
        acc += w1 * r1;
        acc += w0 * r2;
        at_byte(rc, ((unsigned)Y * (unsigned)nc + (unsigned)X) * (unsigned)sizeof(T)) = acc;
    }
}

template <typename T, bool ZERO, class RT>
__device__ __forceinline__ void rows_rbgs_restrict_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                        T* __restrict__ e_out, T* __restrict__ rc, int n, int x0,
                                                        int y0, T a, T diag, T invdiag) {
    __shared__ T se[RT::N];
    __shared__ T sr[RT::N];
    RRStage<T, RT> st;
    rr_load<T, ZERO, RT>(st, r, e_in, n, x0, y0);
    rr_run<T, RT>(st, se, sr, e_out, rc, n, x0, y0, a, diag, invdiag);
}

// The first launch of a substep's solve from e = 0 with the right-hand side
// of eq. (4) formed in it (guess g = u_{m+1}^k, where the L_h terms cancel):
// r = u_m^{k+1} + dt_m [f^E(u_m^{k+1}) - f^E(u_m^k)] + S F - u_{m+1}^k on the
// region the step reads, the tile's part written to r_out for the later
// kernels, then rr_run as rows_rbgs_restrict_body (ZERO).  The values of a
// separate rhs pass followed by rows_rbgs_restrict_body<T, true, RT>.
template <typename T, class RT, typename FE>
__device__ __forceinline__ void rows_rhs_rbgs_restrict_body(const double* __restrict__ um_new,
                                                            const double* __restrict__ um_old,
                                                            const double* __restrict__ up_old,
                                                            const double* __restrict__ sf, double dtm, bool read_old,
                                                            FE fexp,
                                                            T* __restrict__ r_out, T* __restrict__ e_out,
                                                            T* __restrict__ rc, int n, int x0, int y0, T a, T diag,
                                                            T invdiag) {
    __shared__ T se[RT::N];
    __shared__ T sr[RT::N];
    RRStage<T, RT> st;
#pragma unroll
    for (int i = 0; i < RT::IP; ++i) st.ve[i] = T(0);
    {
        const Region R2 = region(2, 1, 1, x0, y0, n, RT::TX, RT::TY);
        double un[RT::IP], uo[RT::IP], upo[RT::IP], sfv[RT::IP];
        rows_load<RT>(un, um_new, n, x0, y0, R2);
        if (read_old) {  // u_m^k only enters through f^E
            rows_load<RT>(uo, um_old, n, x0, y0, R2);
        } else {
#pragma unroll
            for (int i = 0; i < RT::IP; ++i) uo[i] = 0.0;
        }
        rows_load<RT>(upo, up_old, n, x0, y0, R2);
        rows_load<RT>(sfv, sf, n, x0, y0, R2);
#pragma unroll
        for (int i = 0; i < RT::IP; ++i) {
            const double base = un[i] + dtm * (fexp(un[i]) - fexp(uo[i])) + sfv[i];
            st.vr[i] = T(base - upo[i]);  // zero outside the region: every input loads as zero there
        }
    }
    rows_store<RT>(r_out, n, x0, y0, region(0, 0, 0, x0, y0, n, RT::TX, RT::TY),
                   [&](int, int i) { return st.vr[i]; });
    rr_run<T, RT>(st, se, sr, e_out, rc, n, x0, y0, a, diag, invdiag);
}

// e_in + P ec (linear interpolation) on the tile plus a halo of 2, then one
// red-black step.  MODE 0: result to e_out; 1: u_out = g + result (float64);
// 2: u_out = result.
template <typename T, int MODE, class RT>
__device__ __forceinline__ void rows_prolong_rbgs_body(const T* __restrict__ r, const T* __restrict__ e_in,
                                                       const T* __restrict__ ec, T* __restrict__ e_out, int n, int x0,
                                                       int y0, T a, T invdiag, const double* __restrict__ g,
                                                       double* __restrict__ u_out) {
    constexpr int H = RT::H;
    __shared__ T se[RT::N];
    __shared__ T sr[RT::N];
    __shared__ T sc[RT::ICP * RT::RC * H];  // coarse rows y0/2-2 .., columns x0/2-2 .. (stride H)
    const int nc = (n - 1) / 2;
    const Region R2 = region(2, 0, 0, x0, y0, n, RT::TX, RT::TY);
    const Region R1 = region(1, 0, 0, x0, y0, n, RT::TX, RT::TY);
    const Region T0 = region(0, 0, 0, x0, y0, n, RT::TX, RT::TY);
    double vg[RT::IP];
    {
        T ve[RT::IP], vr[RT::IP], vc[RT::ICP];
        rows_load<RT>(ve, e_in, n, x0, y0, R2);
        rows_load<RT>(vr, r, n, x0, y0, R1);
        {
            // coarse box: columns x0/2-2 + cc, rows y0/2-2 + cr (zero outside 0..nc-1)
            const int cc = threadIdx.x % H, cr0 = threadIdx.x / H;
            const int X = x0 / 2 - 2 + cc;
            const bool xok = X >= 0 && X < nc;
#pragma unroll
            for (int i = 0; i < RT::ICP; ++i) {
                const int cr = cr0 + i * RT::RC;
                const int Y = y0 / 2 - 2 + cr;
                T x = T(0);
                if (xok && cr < RT::CROWS && Y >= 0 && Y < nc)
                    x = at_byte(ec, ((unsigned)Y * (unsigned)nc + (unsigned)X) * (unsigned)sizeof(T));
                vc[i] = x;
            }
        }
        if (MODE == 1) {
            const int c = threadIdx.x % RT::LPR, j = threadIdx.x / RT::LPR;
            const bool cok = c >= T0.clo && c <= T0.chi;
            const unsigned rowb = (unsigned)n * sizeof(double);
            const unsigned off0 = (unsigned)(y0 - 3 + j) * rowb + (unsigned)(x0 - 3 + c) * (unsigned)sizeof(double);
#pragma unroll
            for (int i = 0; i < RT::IP; ++i) {
                const int row = j + i * RT::RP;
                double x = 0.0;
                if (cok && row >= T0.rlo && row <= T0.rhi) x = at_byte(g, off0 + (unsigned)(i * RT::RP) * rowb);
                vg[i] = x;
            }
        }
        rows_store_lds<RT>(se, ve);
        rows_store_lds<RT>(sr, vr);
#pragma unroll
        for (int i = 0; i < RT::ICP; ++i) sc[threadIdx.x + i * kThreads] = vc[i];
    }
    __syncthreads();
    {
        // coarse-grid correction on the halo-2 region.  Fine x = x0 - 3 + c is
        // odd for even c (one coarse point, column c/2 of sc) and even for odd c
        // (mean of columns (c-1)/2 and (c+1)/2); rows likewise (RP is even, so
        // the row parity is the thread's).
        const int c = threadIdx.x % RT::LPR, j = threadIdx.x / RT::LPR;
        const bool xodd = !(c & 1), yodd = !(j & 1);
        const T wx0 = xodd ? T(1) : T(0.5), wx1 = xodd ? T(0) : T(0.5);
        const T wy0 = yodd ? T(1) : T(0.5), wy1 = yodd ? T(0) : T(0.5);
        const int ix = xodd ? c / 2 : (c - 1) / 2;
        const int iy = yodd ? j / 2 : (j - 1) / 2;
        const int cb = iy * H + ix;
        T v[RT::IP];
        bool w[RT::IP];
#pragma unroll
        for (int i = 0; i < RT::IP; ++i) w[i] = false;
        rows_plain<RT>(R2, [&](int k, int i) {
            const int b = cb + i * (RT::RP / 2) * H;
            T acc = wy0 * (wx0 * sc[b] + wx1 * sc[b + 1]);
            acc += wy1 * (wx0 * sc[b + H] + wx1 * sc[b + H + 1]);
            v[i] = se[k] + acc;
            w[i] = true;
        });
#pragma unroll
        for (int i = 0; i < RT::IP; ++i)
            if (w[i]) se[threadIdx.x + i * kThreads] = v[i];
    }
    __syncthreads();
    rows_colour<RT>(se, sr, 0, x0, y0, R1, a, invdiag);
    __syncthreads();
    rows_colour<RT>(se, sr, 1, x0, y0, T0, a, invdiag);
    __syncthreads();
    if (MODE == 0) {
        rows_store<RT>(e_out, n, x0, y0, T0, [&](int k, int) { return se[k]; });
    } else {
        rows_store<RT>(u_out, n, x0, y0, T0, [&](int k, int i) {
            return MODE == 1 ? vg[i] + (double)se[k] : (double)se[k];
        });
    }
}

}  // namespace
}  // namespace isdc
