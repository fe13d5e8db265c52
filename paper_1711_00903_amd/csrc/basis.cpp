// basis.cpp -- quadrature rules and 1-D operator tables of degree N (Notation
// table; eqs. interpolationOps and derivativeOps), computed on the host.
//
// Nodes: Newton's method on Legendre polynomials evaluated by the three-term
// recurrence.  Gauss-Legendre nodes are the roots of P_n (weights
// 2 / ((1 - x^2) P_n'(x)^2)); the interior Gauss-Lobatto-Legendre nodes are the
// roots of q(x) = (1 - x^2) P_N'(x), whose derivative is -N(N+1) P_N(x) by
// Legendre's equation (weights 2 / (N (N+1) P_N(x)^2)).
//
// Tables: barycentric Lagrange formulas (Berrut & Trefethen, SIAM Review 46,
// 2004).  With barycentric weights lambda_i = 1 / prod_{m != i}(x_i - x_m):
//   interpolation  l_i(y) = (lambda_i / (y - x_i)) / sum_m lambda_m / (y - x_m),
//   differentiation at the nodes D_ai = (lambda_i / lambda_a) / (x_a - x_i),
//   a != i, and D_aa = -sum_{i != a} D_ai (rows of D annihilate constants).
#include <cmath>
#include <cstring>
#include <utility>

#include "launch.hpp"

namespace fem {

namespace {

void legendre_pair(int n, double x, double *p, double *dp)
{
    // P_n and P_n' by the recurrence; P_n' from (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    // is singular at +-1, so carry the derivative recurrence instead:
    // P'_{k+1} = (k+1) P_k + x P'_k.
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { *p = 1.0; *dp = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        const double p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        const double d2 = (k + 1) * p1 + x * d1;
        p0 = p1; p1 = p2;
        d0 = d1; d1 = d2;
    }
    *p = p1;
    *dp = d1;
}

void sort_nodes(int n, double *r, double *w)
{
    for (int a = 0; a < n; ++a) {
        int best = a;
        for (int b = a + 1; b < n; ++b)
            if (r[b] < r[best]) best = b;
        std::swap(r[a], r[best]);
        std::swap(w[a], w[best]);
    }
}

void barycentric_weights(int n, const double *x, double *lam)
{
    for (int i = 0; i < n; ++i) {
        double p = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != i) p *= (x[i] - x[m]);
        lam[i] = 1.0 / p;
    }
}

// out[a][i] = l_i(y_a) for the Lagrange basis of nodes x (n of them), at ny points.
void interp_matrix(int n, const double *x, int ny, const double *y, double *out)
{
    double lam[32];
    barycentric_weights(n, x, lam);
    for (int a = 0; a < ny; ++a) {
        int hit = -1;
        for (int i = 0; i < n; ++i)
            if (y[a] == x[i]) hit = i;
        if (hit >= 0) {
            for (int i = 0; i < n; ++i) out[a * n + i] = (i == hit) ? 1.0 : 0.0;
            continue;
        }
        double den = 0.0;
        for (int i = 0; i < n; ++i) den += lam[i] / (y[a] - x[i]);
        for (int i = 0; i < n; ++i) out[a * n + i] = (lam[i] / (y[a] - x[i])) / den;
    }
}

// out[a][i] = l_i'(x_a) at the nodes themselves.
void diff_matrix(int n, const double *x, double *out)
{
    double lam[32];
    barycentric_weights(n, x, lam);
    for (int a = 0; a < n; ++a) {
        double diag = 0.0;
        for (int i = 0; i < n; ++i) {
            if (i == a) continue;
            const double v = (lam[i] / lam[a]) / (x[a] - x[i]);
            out[a * n + i] = v;
            diag -= v;
        }
        out[a * n + a] = diag;
    }
}

}  // namespace

int gauss_legendre(int n, double *r, double *w)
{
    if (n < 1 || n > 32) return 1;
    for (int i = 0; i < n; ++i) {
        // Tricomi's first-order estimate of the i-th root, then Newton.
        const double th = M_PI * (4.0 * i + 3.0) / (4.0 * n + 2.0);
        double x = std::cos(th) * (1.0 - (n - 1.0) / (8.0 * n * n * n));
        for (int it = 0; it < 64; ++it) {
            double p, dp;
            legendre_pair(n, x, &p, &dp);
            const double step = p / dp;
            x -= step;
            if (std::fabs(step) <= 4e-16 * std::fabs(x) + 1e-300) break;
        }
        double p, dp;
        legendre_pair(n, x, &p, &dp);
        r[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    sort_nodes(n, r, w);
    return 0;
}

int gauss_lobatto(int N, double *r, double *w)
{
    if (N < 1 || N > 31) return 1;
    const double nn = N * (N + 1.0);
    r[0] = -1.0;
    r[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = std::cos(M_PI * (N - i) / N);   // Chebyshev-Lobatto start, ascending
        for (int it = 0; it < 64; ++it) {
            double p, dp;
            legendre_pair(N, x, &p, &dp);
            const double q = (1.0 - x * x) * dp;   // vanishes at the GLL nodes
            const double dq = -nn * p;
            const double step = q / dq;
            x -= step;
            if (std::fabs(step) <= 4e-16) break;
        }
        r[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double p, dp;
        legendre_pair(N, r[i], &p, &dp);
        w[i] = 2.0 / (nn * p * p);
    }
    sort_nodes(N + 1, r, w);
    return 0;
}

int basis_tables(int N, double *r_gll, double *w_gll, double *r_gl, double *w_gl, double *I1d,
                 double *D1d, double *Dgl)
{
    if (N < 1 || N > kMaxN) return 1;
    const int nq = N + 1, ng = N + 2;
    double rq[kMaxN + 2], wq[kMaxN + 2], rg[kMaxN + 2], wg[kMaxN + 2];
    if (gauss_lobatto(N, rq, wq) || gauss_legendre(ng, rg, wg)) return 1;
    if (r_gll) std::memcpy(r_gll, rq, sizeof(double) * nq);
    if (w_gll) std::memcpy(w_gll, wq, sizeof(double) * nq);
    if (r_gl) std::memcpy(r_gl, rg, sizeof(double) * ng);
    if (w_gl) std::memcpy(w_gl, wg, sizeof(double) * ng);
    if (I1d) interp_matrix(nq, rq, ng, rg, I1d);
    if (D1d) diff_matrix(nq, rq, D1d);
    if (Dgl) diff_matrix(ng, rg, Dgl);
    return 0;
}

}  // namespace fem
