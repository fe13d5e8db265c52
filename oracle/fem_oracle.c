/*
 * fem_oracle.c -- plain, slow, FP64 CPU oracle for the hexahedral
 * tensor-product operators BP1.0 (mass), BP3.5 (collocated stiffness) and
 * BP3.0 (de-aliased stiffness) of Swirydowicz, Chalmers, Karakus & Warburton,
 * "Acceleration of tensor-product operations for high-order finite element
 * methods" (arXiv 1711.00903).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference against
 * which the GPU library is checked.  Only the test-suite, the package smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * Every function below cites the passage of the paper it follows.  Readings
 * where the paper is garbled or ambiguous:
 *   - The 1-D differentiation matrices are printed as l_i(r_a); read as the
 *     derivatives l_i'(r_a) (and l~_i'(r~_a)), as the operators D^r, D^s, D^t
 *     of eq. (derivativeOps) require.
 *   - The metric tensor is printed as |J| J^T J with J "from element to
 *     reference cube".  Read with J = dx/dr (reference -> physical):
 *     G = w * detJ * J^{-1} J^{-T}, i.e. G_ab = w detJ sum_d dr_a/dx_d dr_b/dx_d.
 *     The quadrature weights w_a w_b w_c are folded into G and into the
 *     scaled Jacobian (eq. Gdef and the J^e definitions).
 *   - Interpolation (Alg. 1) and projection (Alg. 2) are pure I and I^T; the
 *     scaled Jacobian is applied exactly once, in the mass operator (Alg. 3).
 *   - In the output line of Alg. 4/5 the third transposed term uses rqt.
 *   - The BP3.0 lambda term uses the interpolated field at the GL nodes and is
 *     projected with the stiffness term: I^T (D~^T G D~ + lambda J) I.
 *
 * Node ordering: node (i,j,k) of an element, i along r (fastest), j along s,
 * k along t, is stored at i + Nq*j + Nq*Nq*k.  Geometric factors are stored
 * [E][6][Npq] in the order rr, rs, rt, ss, st, tt; scaled Jacobians [E][Npq].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXN 15
#define ORA_MAXQ (ORA_MAXN + 2)

/* ---------------------------------------------------------------------------
 * Legendre polynomials (textbook three-term recurrence).
 *   P_0 = 1, P_1 = x, (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}.
 * Returns P_n(x); *dp = P_n'(x) via the same recurrence differentiated:
 *   P'_{k+1} = P'_{k-1} + (2k+1) P_k.
 * ------------------------------------------------------------------------- */
static double legendre(int n, double x, double *dp)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (n == 0) { if (dp) *dp = 0.0; return 1.0; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    if (dp) *dp = d1;
    return p1;
}

static void sort_ascending(int n, double *r, double *w)
{
    for (int a = 1; a < n; ++a)
        for (int b = a; b > 0 && r[b] < r[b - 1]; --b) {
            double t = r[b]; r[b] = r[b - 1]; r[b - 1] = t;
            t = w[b]; w[b] = w[b - 1]; w[b - 1] = t;
        }
}

/* n-point Gauss-Legendre rule: nodes are the roots of P_n, weights
 * 2 / ((1 - x^2) P_n'(x)^2).  Used for the N+2 GL points of BP1.0 and BP3.0
 * (Notation table, glNq = N+2). */
int ora_gl(int n, double *r, double *w)
{
    if (n < 1 || n > ORA_MAXQ + 8) return 1;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double d, p = legendre(n, x, &d);
            double dx = p / d;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        double d;
        legendre(n, x, &d);
        r[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * d * d);
    }
    sort_ascending(n, r, w);
    return 0;
}

/* (N+1)-point Gauss-Lobatto-Legendre rule: nodes -1, +1 and the roots of
 * P_N', weights 2 / (N (N+1) P_N(x)^2).  These are the interpolation nodes of
 * the element basis (Problem description section). */
int ora_gll(int N, double *r, double *w)
{
    if (N < 1 || N > ORA_MAXQ + 8) return 1;
    const double c = N * (N + 1.0);
    r[0] = -1.0; r[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double d1, p = legendre(N, x, &d1);
            /* Legendre's equation: (1-x^2) P'' = 2 x P' - N(N+1) P */
            double d2 = (2.0 * x * d1 - c * p) / (1.0 - x * x);
            double dx = d1 / d2;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        r[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double p = legendre(N, r[i], NULL);
        w[i] = 2.0 / (c * p * p);
    }
    sort_ascending(N + 1, r, w);
    return 0;
}

/* Lagrange polynomial l_i of the nodes x[0..n-1], evaluated at y, straight
 * from its product definition. */
static double lagrange(int n, const double *x, int i, double y)
{
    double v = 1.0;
    for (int m = 0; m < n; ++m)
        if (m != i) v *= (y - x[m]) / (x[i] - x[m]);
    return v;
}

/* Derivative of l_i at y by the product rule applied to that definition:
 * l_i'(y) = sum_{m != i} 1/(x_i - x_m) prod_{p != i, m} (y - x_p)/(x_i - x_p). */
static double lagrange_deriv(int n, const double *x, int i, double y)
{
    double s = 0.0;
    for (int m = 0; m < n; ++m) {
        if (m == i) continue;
        double t = 1.0 / (x[i] - x[m]);
        for (int p = 0; p < n; ++p)
            if (p != i && p != m) t *= (y - x[p]) / (x[i] - x[p]);
        s += t;
    }
    return s;
}

/* 1-D tables of the Notation table and eqs. (interpolationOps),
 * (derivativeOps):
 *   I1d[a][i] = l_i(r~_a)     (N+2) x (N+1), GLL basis at the GL nodes
 *   D1d[a][i] = l_i'(r_a)     (N+1) x (N+1), GLL basis derivative at GLL nodes
 *   Dgl[a][b] = l~_b'(r~_a)   (N+2) x (N+2), GL basis derivative at GL nodes
 * all row-major.  Also returns the GLL and GL nodes and weights. */
int ora_tables(int N, double *rgll, double *wgll, double *rgl, double *wgl,
               double *I1d, double *D1d, double *Dgl)
{
    if (N < 1 || N > ORA_MAXN) return 1;
    const int nq = N + 1, ng = N + 2;
    if (ora_gll(N, rgll, wgll) || ora_gl(ng, rgl, wgl)) return 1;
    for (int a = 0; a < ng; ++a)
        for (int i = 0; i < nq; ++i)
            I1d[a * nq + i] = lagrange(nq, rgll, i, rgl[a]);
    for (int a = 0; a < nq; ++a)
        for (int i = 0; i < nq; ++i)
            D1d[a * nq + i] = lagrange_deriv(nq, rgll, i, rgll[a]);
    for (int a = 0; a < ng; ++a)
        for (int b = 0; b < ng; ++b)
            Dgl[a * ng + b] = lagrange_deriv(ng, rgl, b, rgl[a]);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Geometry (Problem description section): each element is the image of the
 * bi-unit reference cube under the trilinear map through its 8 vertices,
 *   x(r,s,t) = sum_{a,b,c in {0,1}} X_{abc} phi_a(r) phi_b(s) phi_c(t),
 *   phi_0(z) = (1-z)/2, phi_1(z) = (1+z)/2,
 * vertex (a,b,c) stored at X[e][a + 2b + 4c][0..2].
 * ------------------------------------------------------------------------- */
static double phi(int a, double z) { return a ? 0.5 * (1.0 + z) : 0.5 * (1.0 - z); }
static double dphi(int a) { return a ? 0.5 : -0.5; }

/* Jacobian J[d][al] = d x_d / d r_al at (r,s,t). */
static void trilinear_jacobian(const double *X, double r, double s, double t,
                               double J[3][3])
{
    for (int d = 0; d < 3; ++d)
        for (int al = 0; al < 3; ++al) J[d][al] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double *v = X + 3 * (a + 2 * b + 4 * c);
                double gr = dphi(a) * phi(b, s) * phi(c, t);
                double gs = phi(a, r) * dphi(b) * phi(c, t);
                double gt = phi(a, r) * phi(b, s) * dphi(c);
                for (int d = 0; d < 3; ++d) {
                    J[d][0] += v[d] * gr;
                    J[d][1] += v[d] * gs;
                    J[d][2] += v[d] * gt;
                }
            }
}

static void trilinear_point(const double *X, double r, double s, double t, double x[3])
{
    x[0] = x[1] = x[2] = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const double *v = X + 3 * (a + 2 * b + 4 * c);
                double p = phi(a, r) * phi(b, s) * phi(c, t);
                for (int d = 0; d < 3; ++d) x[d] += v[d] * p;
            }
}

static double det3(double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Inverse of a 3x3 matrix by Gauss-Jordan elimination with partial pivoting.
 * Returns 1 if singular. */
static int inverse3(double A[3][3], double B[3][3])
{
    double M[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) { M[i][j] = A[i][j]; M[i][3 + j] = (i == j); }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int i = col + 1; i < 3; ++i)
            if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
        if (M[piv][col] == 0.0) return 1;
        if (piv != col)
            for (int j = 0; j < 6; ++j) { double t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
        double inv = 1.0 / M[col][col];
        for (int j = 0; j < 6; ++j) M[col][j] *= inv;
        for (int i = 0; i < 3; ++i) {
            if (i == col) continue;
            double f = M[i][col];
            for (int j = 0; j < 6; ++j) M[i][j] -= f * M[col][j];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = M[i][3 + j];
    return 0;
}

/* Geometric factors at the nodes of a tensor rule with nq points per
 * direction (GLL: quad = 0, nq = N+1, as in BP3.5; GL: quad = 1, nq = N+2, as
 * in BP1.0 and BP3.0).  For node (a,b,c):
 *   wJ  = w_a w_b w_c |J|                                (the J^e diagonals)
 *   G   = w_a w_b w_c |J| J^{-1} J^{-T}, 6 entries rr, rs, rt, ss, st, tt
 * G may be NULL (mass only) and wJ may be NULL.  Returns the number of nodes
 * with detJ <= 0 (0 on a valid mesh), or -1 on bad arguments. */
int64_t ora_geometry(int N, int64_t E, int quad, const double *X, double *G, double *wJ)
{
    if (N < 1 || N > ORA_MAXN || E < 0 || (quad != 0 && quad != 1)) return -1;
    double r[ORA_MAXQ], w[ORA_MAXQ];
    int nq = quad ? N + 2 : N + 1;
    if (quad) ora_gl(nq, r, w); else ora_gll(N, r, w);
    const int64_t npq = (int64_t)nq * nq * nq;
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+:bad)
    for (int64_t e = 0; e < E; ++e) {
        const double *Xe = X + 24 * e;
        for (int c = 0; c < nq; ++c)
            for (int b = 0; b < nq; ++b)
                for (int a = 0; a < nq; ++a) {
                    int64_t n = a + nq * (b + (int64_t)nq * c);
                    double J[3][3], Ji[3][3];
                    trilinear_jacobian(Xe, r[a], r[b], r[c], J);
                    double dJ = det3(J);
                    if (!(dJ > 0.0)) ++bad;
                    double ww = w[a] * w[b] * w[c];
                    if (wJ) wJ[e * npq + n] = ww * dJ;
                    if (G) {
                        if (inverse3(J, Ji)) { ++bad; continue; }
                        double g[3][3];
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q) {
                                double sum = 0.0;
                                for (int d = 0; d < 3; ++d) sum += Ji[p][d] * Ji[q][d];
                                g[p][q] = ww * dJ * sum;
                            }
                        double *Ge = G + 6 * npq * e;
                        Ge[0 * npq + n] = g[0][0];
                        Ge[1 * npq + n] = g[0][1];
                        Ge[2 * npq + n] = g[0][2];
                        Ge[3 * npq + n] = g[1][1];
                        Ge[4 * npq + n] = g[1][2];
                        Ge[5 * npq + n] = g[2][2];
                    }
                }
    }
    return bad;
}

/* Physical coordinates [E][Npq][3] of the element's tensor nodes (GLL if
 * quad == 0, GL if quad == 1) under the trilinear map. */
int ora_node_coords(int N, int64_t E, int quad, const double *X, double *xyz)
{
    if (N < 1 || N > ORA_MAXN || E < 0) return 1;
    double r[ORA_MAXQ], w[ORA_MAXQ];
    int nq = quad ? N + 2 : N + 1;
    if (quad) ora_gl(nq, r, w); else ora_gll(N, r, w);
    const int64_t npq = (int64_t)nq * nq * nq;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e)
        for (int c = 0; c < nq; ++c)
            for (int b = 0; b < nq; ++b)
                for (int a = 0; a < nq; ++a) {
                    int64_t n = a + nq * (b + (int64_t)nq * c);
                    trilinear_point(X + 24 * e, r[a], r[b], r[c], xyz + 3 * (e * npq + n));
                }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Operators, element by element (the global operators are block diagonal:
 * no coupling between elements).  Arrays q[c][b][a] are indexed with a (r)
 * fastest.  nq = N+1 GLL points, ng = N+2 GL points.
 * ------------------------------------------------------------------------- */

/* Alg. 1 (Interpolation GLL -> GL): three one-direction contractions with
 * I1d, in the order s (b), r (a), t (c).  q: nq^3 -> out: ng^3.
 * t1 holds nq*ng*nq, t2 holds nq*ng*ng values. */
static void interpolate(int nq, int ng, const double *I, const double *q,
                        double *t1, double *t2, double *out)
{
    /* s direction: t1[c][j][a] = sum_b I[j][b] q[c][b][a] */
    for (int c = 0; c < nq; ++c)
        for (int j = 0; j < ng; ++j)
            for (int a = 0; a < nq; ++a) {
                double s = 0.0;
                for (int b = 0; b < nq; ++b) s += I[j * nq + b] * q[(c * nq + b) * nq + a];
                t1[(c * ng + j) * nq + a] = s;
            }
    /* r direction: t2[c][j][i] = sum_a I[i][a] t1[c][j][a] */
    for (int c = 0; c < nq; ++c)
        for (int j = 0; j < ng; ++j)
            for (int i = 0; i < ng; ++i) {
                double s = 0.0;
                for (int a = 0; a < nq; ++a) s += I[i * nq + a] * t1[(c * ng + j) * nq + a];
                t2[(c * ng + j) * ng + i] = s;
            }
    /* t direction: out[k][j][i] = sum_c I[k][c] t2[c][j][i] */
    for (int k = 0; k < ng; ++k)
        for (int j = 0; j < ng; ++j)
            for (int i = 0; i < ng; ++i) {
                double s = 0.0;
                for (int c = 0; c < nq; ++c) s += I[k * nq + c] * t2[(c * ng + j) * ng + i];
                out[(k * ng + j) * ng + i] = s;
            }
}

/* Alg. 2 (Projection GL -> GLL): three contractions with I1d^T, in the order
 * s, r, t.  qt: ng^3 -> out: nq^3.  t1 holds ng*nq*ng, t2 holds ng*nq*nq. */
static void project(int nq, int ng, const double *I, const double *qt,
                    double *t1, double *t2, double *out)
{
    /* s direction: t1[k][b][i] = sum_j I[j][b] qt[k][j][i] */
    for (int k = 0; k < ng; ++k)
        for (int b = 0; b < nq; ++b)
            for (int i = 0; i < ng; ++i) {
                double s = 0.0;
                for (int j = 0; j < ng; ++j) s += I[j * nq + b] * qt[(k * ng + j) * ng + i];
                t1[(k * nq + b) * ng + i] = s;
            }
    /* r direction: t2[k][b][a] = sum_i I[i][a] t1[k][b][i] */
    for (int k = 0; k < ng; ++k)
        for (int b = 0; b < nq; ++b)
            for (int a = 0; a < nq; ++a) {
                double s = 0.0;
                for (int i = 0; i < ng; ++i) s += I[i * nq + a] * t1[(k * nq + b) * ng + i];
                t2[(k * nq + b) * nq + a] = s;
            }
    /* t direction: out[c][b][a] = sum_k I[k][c] t2[k][b][a] */
    for (int c = 0; c < nq; ++c)
        for (int b = 0; b < nq; ++b)
            for (int a = 0; a < nq; ++a) {
                double s = 0.0;
                for (int k = 0; k < ng; ++k) s += I[k * nq + c] * t2[(k * nq + b) * nq + a];
                out[(c * nq + b) * nq + a] = s;
            }
}

/* Collocated screened-Poisson action on one element with n points per
 * direction (Alg. 4 for BP3.5 with the GLL D1d; the inner part of Alg. 5 for
 * BP3.0 with the GL Dgl):
 *   qr = sum_m D[i][m] q[k][j][m], qs = sum_m D[j][m] q[k][m][i],
 *   qt = sum_m D[k][m] q[m][j][i];
 *   (rqr, rqs, rqt) = G (qr, qs, qt) with G symmetric;
 *   out[k][j][i] = sum_m D[m][i] rqr[k][j][m] + D[m][j] rqs[k][m][i]
 *                + D[m][k] rqt[m][j][i]  (+ lambda * wJ * q).
 * G points at the element's 6 factor arrays of n^3 values each. */
static void stiffness_collocated(int n, const double *D, const double *G, const double *wJ,
                                 double lambda, const double *q,
                                 double *rqr, double *rqs, double *rqt, double *out)
{
    const int64_t np = (int64_t)n * n * n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int64_t id = (k * n + j) * n + i;
                double qr = 0.0, qs = 0.0, qt = 0.0;
                for (int m = 0; m < n; ++m) {
                    qr += D[i * n + m] * q[(k * n + j) * n + m];
                    qs += D[j * n + m] * q[(k * n + m) * n + i];
                    qt += D[k * n + m] * q[(m * n + j) * n + i];
                }
                double grr = G[0 * np + id], grs = G[1 * np + id], grt = G[2 * np + id];
                double gss = G[3 * np + id], gst = G[4 * np + id], gtt = G[5 * np + id];
                rqr[id] = grr * qr + grs * qs + grt * qt;
                rqs[id] = grs * qr + gss * qs + gst * qt;
                rqt[id] = grt * qr + gst * qs + gtt * qt;
            }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int64_t id = (k * n + j) * n + i;
                double s = 0.0;
                for (int m = 0; m < n; ++m) {
                    s += D[m * n + i] * rqr[(k * n + j) * n + m];
                    s += D[m * n + j] * rqs[(k * n + m) * n + i];
                    s += D[m * n + k] * rqt[(m * n + j) * n + i];
                }
                if (lambda != 0.0) s += lambda * wJ[id] * q[id];
                out[id] = s;
            }
}

#define ORA_SCRATCH(ng) ((int64_t)(ng) * (ng) * (ng))

/* BP1.0, Alg. 3: y^e = I^T J^e I u^e (eq. massQuad; M^e = I^T J^e I).
 * wJ: [E][ng^3] GL-scaled Jacobians.  If accumulate, y += result. */
int ora_bp10(int N, int64_t E, const double *I1d, const double *wJ, const double *u,
             double *y, int accumulate)
{
    if (N < 1 || N > ORA_MAXN || E < 0) return 1;
    const int nq = N + 1, ng = N + 2;
    const int64_t np = (int64_t)nq * nq * nq, npg = (int64_t)ng * ng * ng;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 5 * ORA_SCRATCH(ng));
        double *t1 = buf, *t2 = buf + npg, *qg = buf + 2 * npg, *res = buf + 3 * npg;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            interpolate(nq, ng, I1d, u + e * np, t1, t2, qg);
            for (int64_t n = 0; n < npg; ++n) qg[n] *= wJ[e * npg + n];
            project(nq, ng, I1d, qg, t1, t2, res);
            for (int64_t n = 0; n < np; ++n)
                y[e * np + n] = accumulate ? y[e * np + n] + res[n] : res[n];
        }
        free(buf);
    }
    return 0;
}

/* BP3.5, Alg. 4: y^e = D^T G^e D u^e + lambda J^e u^e (GLL collocation,
 * eq. stiffQuad).  G: [E][6][nq^3]; wJ: [E][nq^3] (GLL), may be NULL iff
 * lambda == 0. */
int ora_bp35(int N, int64_t E, const double *D1d, const double *G, const double *wJ,
             double lambda, const double *u, double *y, int accumulate)
{
    if (N < 1 || N > ORA_MAXN || E < 0 || (lambda != 0.0 && !wJ)) return 1;
    const int nq = N + 1;
    const int64_t np = (int64_t)nq * nq * nq;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 4 * np);
        double *rqr = buf, *rqs = buf + np, *rqt = buf + 2 * np, *res = buf + 3 * np;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            stiffness_collocated(nq, D1d, G + 6 * np * e, wJ ? wJ + np * e : NULL, lambda,
                                 u + np * e, rqr, rqs, rqt, res);
            for (int64_t n = 0; n < np; ++n)
                y[e * np + n] = accumulate ? y[e * np + n] + res[n] : res[n];
        }
        free(buf);
    }
    return 0;
}

/* BP3.0, Alg. 5: y^e = I^T (D~^T G^e D~ + lambda J^e) I u^e (GL quadrature,
 * eq. stiffQuad2).  G: [E][6][ng^3] at GL nodes; wJ: [E][ng^3] (GL), may be
 * NULL iff lambda == 0. */
int ora_bp30(int N, int64_t E, const double *I1d, const double *Dgl, const double *G,
             const double *wJ, double lambda, const double *u, double *y, int accumulate)
{
    if (N < 1 || N > ORA_MAXN || E < 0 || (lambda != 0.0 && !wJ)) return 1;
    const int nq = N + 1, ng = N + 2;
    const int64_t np = (int64_t)nq * nq * nq, npg = (int64_t)ng * ng * ng;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 8 * npg);
        double *t1 = buf, *t2 = buf + npg, *qg = buf + 2 * npg, *rqr = buf + 3 * npg;
        double *rqs = buf + 4 * npg, *rqt = buf + 5 * npg, *ag = buf + 6 * npg, *res = buf + 7 * npg;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            interpolate(nq, ng, I1d, u + e * np, t1, t2, qg);
            stiffness_collocated(ng, Dgl, G + 6 * npg * e, wJ ? wJ + npg * e : NULL, lambda,
                                 qg, rqr, rqs, rqt, ag);
            project(nq, ng, I1d, ag, t1, t2, res);
            for (int64_t n = 0; n < np; ++n)
                y[e * np + n] = accumulate ? y[e * np + n] + res[n] : res[n];
        }
        free(buf);
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * The residual of the CG workload in extended precision.
 *
 * ||b - (S + lambda M) x||^2 and ||b||^2 over E elements, with S the BP3.5
 * stiffness (Alg. 4, eq. stiffQuad) and M the BP1.0 mass (Alg. 3, eq.
 * massQuad), every product and sum taken in long double (64-bit significand
 * on x86-64) on the FP64 inputs as stored.  Near the rounding floor of the
 * CG workload an FP64 evaluation of b - Ax carries rounding of the size of the
 * residual itself; this one measures the residual of the stored x.
 * The contractions are those of interpolate / project / stiffness_collocated
 * above, in the same order.
 * ------------------------------------------------------------------------- */
typedef long double ora_ld;

static void interpolate_ld(int nq, int ng, const double *I, const ora_ld *q, ora_ld *t1, ora_ld *t2,
                           ora_ld *out)
{
    for (int c = 0; c < nq; ++c)
        for (int j = 0; j < ng; ++j)
            for (int a = 0; a < nq; ++a) {
                ora_ld s = 0.0L;
                for (int b = 0; b < nq; ++b) s += (ora_ld)I[j * nq + b] * q[(c * nq + b) * nq + a];
                t1[(c * ng + j) * nq + a] = s;
            }
    for (int c = 0; c < nq; ++c)
        for (int j = 0; j < ng; ++j)
            for (int i = 0; i < ng; ++i) {
                ora_ld s = 0.0L;
                for (int a = 0; a < nq; ++a) s += (ora_ld)I[i * nq + a] * t1[(c * ng + j) * nq + a];
                t2[(c * ng + j) * ng + i] = s;
            }
    for (int k = 0; k < ng; ++k)
        for (int j = 0; j < ng; ++j)
            for (int i = 0; i < ng; ++i) {
                ora_ld s = 0.0L;
                for (int c = 0; c < nq; ++c) s += (ora_ld)I[k * nq + c] * t2[(c * ng + j) * ng + i];
                out[(k * ng + j) * ng + i] = s;
            }
}

static void project_ld(int nq, int ng, const double *I, const ora_ld *qt, ora_ld *t1, ora_ld *t2, ora_ld *out)
{
    for (int k = 0; k < ng; ++k)
        for (int b = 0; b < nq; ++b)
            for (int i = 0; i < ng; ++i) {
                ora_ld s = 0.0L;
                for (int j = 0; j < ng; ++j) s += (ora_ld)I[j * nq + b] * qt[(k * ng + j) * ng + i];
                t1[(k * nq + b) * ng + i] = s;
            }
    for (int k = 0; k < ng; ++k)
        for (int b = 0; b < nq; ++b)
            for (int a = 0; a < nq; ++a) {
                ora_ld s = 0.0L;
                for (int i = 0; i < ng; ++i) s += (ora_ld)I[i * nq + a] * t1[(k * nq + b) * ng + i];
                t2[(k * nq + b) * nq + a] = s;
            }
    for (int c = 0; c < nq; ++c)
        for (int b = 0; b < nq; ++b)
            for (int a = 0; a < nq; ++a) {
                ora_ld s = 0.0L;
                for (int k = 0; k < ng; ++k) s += (ora_ld)I[k * nq + c] * t2[(k * nq + b) * nq + a];
                out[(c * nq + b) * nq + a] = s;
            }
}

static void stiffness_ld(int n, const double *D, const double *G, const ora_ld *q, ora_ld *rqr, ora_ld *rqs,
                         ora_ld *rqt, ora_ld *out)
{
    const int64_t np = (int64_t)n * n * n;
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int64_t id = (k * n + j) * n + i;
                ora_ld qr = 0.0L, qs = 0.0L, qt = 0.0L;
                for (int m = 0; m < n; ++m) {
                    qr += (ora_ld)D[i * n + m] * q[(k * n + j) * n + m];
                    qs += (ora_ld)D[j * n + m] * q[(k * n + m) * n + i];
                    qt += (ora_ld)D[k * n + m] * q[(m * n + j) * n + i];
                }
                ora_ld grr = G[0 * np + id], grs = G[1 * np + id], grt = G[2 * np + id];
                ora_ld gss = G[3 * np + id], gst = G[4 * np + id], gtt = G[5 * np + id];
                rqr[id] = grr * qr + grs * qs + grt * qt;
                rqs[id] = grs * qr + gss * qs + gst * qt;
                rqt[id] = grt * qr + gst * qs + gtt * qt;
            }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                int64_t id = (k * n + j) * n + i;
                ora_ld s = 0.0L;
                for (int m = 0; m < n; ++m) {
                    s += (ora_ld)D[m * n + i] * rqr[(k * n + j) * n + m];
                    s += (ora_ld)D[m * n + j] * rqs[(k * n + m) * n + i];
                    s += (ora_ld)D[m * n + k] * rqt[(m * n + j) * n + i];
                }
                out[id] = s;
            }
}

/* Returns 0 and writes rr_bb[0] = ||b - A x||^2, rr_bb[1] = ||b||^2.
 * G: BP3.5 factors [E][6][nq^3]; wJ: BP1.0 scaled Jacobians at GL nodes
 * [E][ng^3] (unused when lambda == 0). */
int ora_cg_residual_ld(int N, int64_t E, const double *I1d, const double *D1d, const double *G,
                       const double *wJ, double lambda, const double *x, const double *b, double *rr_bb)
{
    if (N < 1 || N > ORA_MAXN || E < 0 || (lambda != 0.0 && !wJ)) return 1;
    const int nq = N + 1, ng = N + 2;
    const int64_t np = (int64_t)nq * nq * nq, npg = (int64_t)ng * ng * ng;
    ora_ld rr = 0.0L, bb = 0.0L;
#pragma omp parallel reduction(+ : rr, bb)
    {
        ora_ld *buf = (ora_ld *)malloc(sizeof(ora_ld) * (4 * npg + 6 * np));
        ora_ld *t1 = buf, *t2 = buf + npg, *qg = buf + 2 * npg, *mg = buf + 3 * npg;
        ora_ld *q = buf + 4 * npg, *rqr = q + np, *rqs = q + 2 * np, *rqt = q + 3 * np, *ys = q + 4 * np;
        ora_ld *xm = q + 5 * np;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            for (int64_t n = 0; n < np; ++n) q[n] = x[e * np + n];
            stiffness_ld(nq, D1d, G + 6 * np * e, q, rqr, rqs, rqt, ys);
            if (lambda != 0.0) {
                interpolate_ld(nq, ng, I1d, q, t1, t2, qg);
                for (int64_t n = 0; n < npg; ++n) mg[n] = qg[n] * (ora_ld)wJ[e * npg + n];
                project_ld(nq, ng, I1d, mg, t1, t2, xm);
            }
            for (int64_t n = 0; n < np; ++n) {
                ora_ld ax = ys[n] + (lambda != 0.0 ? (ora_ld)lambda * xm[n] : 0.0L);
                ora_ld r = (ora_ld)b[e * np + n] - ax;
                rr += r * r;
                bb += (ora_ld)b[e * np + n] * b[e * np + n];
            }
        }
        free(buf);
    }
    rr_bb[0] = (double)rr;
    rr_bb[1] = (double)bb;
    return 0;
}

int ora_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
