// Collocation nodes and quadrature tables (host only).
//
// Sec. 1 and Sec. 2 (eq. (1)-(2)): nodes of a spectral collocation rule on the
// unit step, the cumulative matrix Q (integrals of the Lagrange polynomials
// from 0 to each node) and the node-to-node matrix S of eq. (2).
//
// Gauss-Legendre nodes are all interior, so the end value of a step needs the
// rule's quadrature weights b_j = integral over [0, 1] of l_j as well.
//
// Method (independent of any other implementation in this repository):
//   * nodes by Newton's method on Legendre polynomials evaluated with the
//     three-term recurrence, in long double, from Chebyshev-type starting
//     values;
//   * Q by expanding each Lagrange polynomial into monomial coefficients
//     (product of linear factors) and integrating term by term, in long
//     double -- exact up to rounding for the degree-(M-1) polynomials here;
//   * S by differencing consecutive rows of Q before rounding to double.
#include <cmath>
#include <vector>
#include <algorithm>

#include "../../include/isdc.h"
#include "tables.h"

namespace isdc {

namespace {

typedef long double ld;

// P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, ld x, ld* p, ld* dp) {
    ld p0 = 1.0L, p1 = x;
    if (n == 0) { *p = 1.0L; *dp = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        ld pk = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = pk;
    }
    *p = p1;
    // (1 - x^2) P_n' = n (P_{n-1} - x P_n), valid for |x| < 1
    *dp = (ld)n * (p0 - x * p1) / (1.0L - x * x);
}

ld newton(ld x, ld (*g)(int, ld, ld*), int n) {
    for (int it = 0; it < 100; ++it) {
        ld dg;
        ld v = g(n, x, &dg);
        ld step = v / dg;
        x -= step;
        if (std::fabs(step) < 1e-19L) break;
    }
    return x;
}

// g(x) = P_n'(x); g' from the Legendre equation (1-x^2) P'' = 2x P' - n(n+1) P.
ld lobatto_g(int n, ld x, ld* dg) {
    ld p, dp;
    legendre(n, x, &p, &dp);
    *dg = (2.0L * x * dp - (ld)n * (n + 1) * p) / (1.0L - x * x);
    return dp;
}

// g(x) = P_M(x) - P_{M-1}(x).
ld radau_g(int M, ld x, ld* dg) {
    ld p1, dp1, p0, dp0;
    legendre(M, x, &p1, &dp1);
    legendre(M - 1, x, &p0, &dp0);
    *dg = dp1 - dp0;
    return p1 - p0;
}

// g(x) = P_M(x).
ld gauss_g(int M, ld x, ld* dg) {
    ld p, dp;
    legendre(M, x, &p, &dp);
    *dg = dp;
    return p;
}

}  // namespace

static bool nodes_ld(int kind, int M, std::vector<ld>& tau) {
    const ld pi = 3.141592653589793238462643383279502884L;
    std::vector<ld> x;
    if (kind == ISDC_NODES_LOBATTO) {
        if (M < 2 || M > ISDC_MAX_M) return false;
        int n = M - 1;
        x.push_back(-1.0L);
        // interior extrema of P_n: start from the Chebyshev-Lobatto points
        for (int i = n - 1; i >= 1; --i) x.push_back(newton(std::cos(pi * i / n), lobatto_g, n));
        x.push_back(1.0L);
    } else if (kind == ISDC_NODES_RADAU_RIGHT) {
        if (M < 1 || M > ISDC_MAX_M) return false;
        // right Radau points: x = 1 and the other roots of P_M - P_{M-1};
        // starting values are the Chebyshev-Radau points cos(2 pi i / (2M - 1))
        for (int i = M - 1; i >= 1; --i) x.push_back(newton(std::cos(2.0L * pi * i / (2 * M - 1)), radau_g, M));
        x.push_back(1.0L);
    } else if (kind == ISDC_NODES_LEGENDRE) {
        if (M < 1 || M > ISDC_MAX_M) return false;
        // roots of P_M from the asymptotic starting values cos(pi (i - 1/4) / (M + 1/2))
        for (int i = 1; i <= M; ++i) x.push_back(newton(std::cos(pi * (i - 0.25L) / (M + 0.5L)), gauss_g, M));
    } else {
        return false;
    }
    std::sort(x.begin(), x.end());
    for (size_t i = 1; i < x.size(); ++i)
        if (!(x[i] > x[i - 1])) return false;  // Newton collapsed onto one root
    tau.resize(x.size());
    for (size_t i = 0; i < x.size(); ++i) tau[i] = (1.0L + x[i]) / 2.0L;
    if (kind == ISDC_NODES_LOBATTO) tau.front() = 0.0L;
    if (kind != ISDC_NODES_LEGENDRE) tau.back() = 1.0L;
    return true;
}

bool tables(int kind, int M, double* tau_out, double* Q_out, double* S_out, double* b_out) {
    std::vector<ld> tau;
    if (!nodes_ld(kind, M, tau)) return false;
    std::vector<ld> Q((size_t)M * M);
    std::vector<ld> coef(M);
    for (int j = 0; j < M; ++j) {
        // monomial coefficients of l_j(s) = prod_{i != j} (s - tau_i) / (tau_j - tau_i)
        std::fill(coef.begin(), coef.end(), 0.0L);
        coef[0] = 1.0L;
        int deg = 0;
        for (int i = 0; i < M; ++i) {
            if (i == j) continue;
            ld inv = 1.0L / (tau[j] - tau[i]);
            for (int k = deg + 1; k >= 1; --k) coef[k] = (coef[k - 1] - tau[i] * coef[k]) * inv;
            coef[0] = -tau[i] * coef[0] * inv;
            ++deg;
        }
        for (int m = 0; m < M; ++m) {
            // integral over [0, tau_m] = sum_k coef_k tau_m^{k+1} / (k+1), Horner form
            ld acc = 0.0L;
            for (int k = M - 1; k >= 0; --k) acc = acc * tau[m] + coef[k] / (k + 1);
            Q[(size_t)m * M + j] = acc * tau[m];
        }
        if (b_out) {  // integral over the whole step [0, 1]
            ld acc = 0.0L;
            for (int k = M - 1; k >= 0; --k) acc += coef[k] / (k + 1);
            b_out[j] = (double)acc;
        }
    }
    for (int m = 0; m < M; ++m) {
        if (tau_out) tau_out[m] = (double)tau[m];
        for (int j = 0; j < M; ++j) {
            ld q = Q[(size_t)m * M + j];
            ld qprev = m > 0 ? Q[(size_t)(m - 1) * M + j] : 0.0L;
            if (Q_out) Q_out[(size_t)m * M + j] = (double)q;
            if (S_out) S_out[(size_t)m * M + j] = (double)(q - qprev);
        }
    }
    return true;
}

}  // namespace isdc
