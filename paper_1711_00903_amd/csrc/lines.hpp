// lines.hpp -- one-dimensional contractions of a whole line held in a
// lane's registers, with uniform (wave-wide) half tables.
//
// Interpolation I (Ng x Nq, Ng = Nq + 1 Gauss points, Nq GLL points) is
// centro-symmetric, I[a][i] = I[Ng-1-a][Nq-1-i]; the derivative matrix D~ on
// the Gauss points is centro-antisymmetric, D~[a][m] = -D~[Ng-1-a][Ng-1-m].
// In even-odd form each product reads the n inputs once as sums and
// differences of mirrored pairs and produces an output and its mirror from
// half tables (the symmetry the BP1.0 optimisation section exploits):
//   I:   Ie[a][m] = (I[a][m] + I[a][Nq-1-m]) / 2   (a < ceil(Ng/2), m < ceil(Nq/2))
//        Io[a][m] = (I[a][m] - I[a][Nq-1-m]) / 2   (a < floor(Ng/2), m < floor(Nq/2))
//   D~:  Dp[a][m] = (D~[a][m] + D~[a][Ng-1-m]) / 2 (a < floor(Ng/2), m < ceil(Ng/2))
//        Dm[a][m] = (D~[a][m] - D~[a][Ng-1-m]) / 2 (a < ceil(Ng/2),  m < floor(Ng/2))
// (a middle column / row, when n is odd, holds the plain entry).  The
// transposes I^T and D~^T use the same half tables with the indices exchanged.
#pragma once

namespace fem {

// Interpolation of one line: x (NQ values) -> y (NG = NQ+1 values).
template <int NQ, class TC>
__device__ __forceinline__ void line_interp(const TC *x, TC *y, const TC (*Ie)[(NQ + 1) / 2],
                                            const TC (*Io)[NQ / 2 > 0 ? NQ / 2 : 1])
{
    constexpr int NG = NQ + 1, QE = NQ / 2, GE = NG / 2, HG = (NG + 1) / 2;
    TC xp[QE > 0 ? QE : 1], xm[QE > 0 ? QE : 1];
#pragma unroll
    for (int m = 0; m < QE; ++m) {
        xp[m] = x[m] + x[NQ - 1 - m];
        xm[m] = x[m] - x[NQ - 1 - m];
    }
#pragma unroll
    for (int a = 0; a < HG; ++a) {
        TC ev = 0, od = 0;
#pragma unroll
        for (int m = 0; m < QE; ++m) ev += Ie[a][m] * xp[m];
        if constexpr (NQ % 2 == 1) ev += Ie[a][QE] * x[QE];
        if (a < GE) {
#pragma unroll
            for (int m = 0; m < QE; ++m) od += Io[a][m] * xm[m];
            y[a] = ev + od;
            y[NG - 1 - a] = ev - od;
        } else {
            y[a] = ev;   // middle Gauss point (NG odd)
        }
    }
}

// Projection of one line: v (NG values) -> w (NQ values), w_i = sum_a I[a][i] v_a.
template <int NQ, class TC>
__device__ __forceinline__ void line_project(const TC *v, TC *w, const TC (*Ie)[(NQ + 1) / 2],
                                             const TC (*Io)[NQ / 2 > 0 ? NQ / 2 : 1])
{
    constexpr int NG = NQ + 1, QE = NQ / 2, GE = NG / 2, HQ = (NQ + 1) / 2;
    TC vp[GE > 0 ? GE : 1], vm[GE > 0 ? GE : 1];
#pragma unroll
    for (int a = 0; a < GE; ++a) {
        vp[a] = v[a] + v[NG - 1 - a];
        vm[a] = v[a] - v[NG - 1 - a];
    }
#pragma unroll
    for (int i = 0; i < HQ; ++i) {
        TC ev = 0, od = 0;
#pragma unroll
        for (int a = 0; a < GE; ++a) ev += Ie[a][i] * vp[a];
        if constexpr (NG % 2 == 1) ev += Ie[GE][i] * v[GE];
        if (i < QE) {
#pragma unroll
            for (int a = 0; a < GE; ++a) od += Io[a][i] * vm[a];
            w[i] = ev + od;
            w[NQ - 1 - i] = ev - od;
        } else {
            w[i] = ev;   // middle GLL point (NQ odd)
        }
    }
}

// Derivative of one Gauss line: y = D~ x (NG values each).  For a < NG/2:
// y_a = M_a + P_a, y_{NG-1-a} = M_a - P_a with P the symmetric part (pair sums,
// and the middle value) and M the antisymmetric part (pair differences).
template <int NG, class TC>
__device__ __forceinline__ void line_deriv(const TC *x, TC *y, const TC (*Dp)[(NG + 1) / 2],
                                           const TC (*Dm)[NG / 2 > 0 ? NG / 2 : 1])
{
    constexpr int GE = NG / 2;
    TC xp[GE > 0 ? GE : 1], xm[GE > 0 ? GE : 1];
#pragma unroll
    for (int m = 0; m < GE; ++m) {
        xp[m] = x[m] + x[NG - 1 - m];
        xm[m] = x[m] - x[NG - 1 - m];
    }
#pragma unroll
    for (int a = 0; a < GE; ++a) {
        TC pp = 0, mm = 0;
#pragma unroll
        for (int m = 0; m < GE; ++m) pp += Dp[a][m] * xp[m];
        if constexpr (NG % 2 == 1) pp += Dp[a][GE] * x[GE];
#pragma unroll
        for (int m = 0; m < GE; ++m) mm += Dm[a][m] * xm[m];
        y[a] = mm + pp;
        y[NG - 1 - a] = mm - pp;
    }
    if constexpr (NG % 2 == 1) {
        TC mm = 0;
#pragma unroll
        for (int m = 0; m < GE; ++m) mm += Dm[GE][m] * xm[m];
        y[GE] = mm;
    }
}

// Transposed derivative of one Gauss line: w = D~^T v.  D~^T is also
// centro-antisymmetric; its half tables are Dm^T (symmetric part) and Dp^T
// (antisymmetric part).
template <int NG, class TC>
__device__ __forceinline__ void line_deriv_t(const TC *v, TC *w, const TC (*Dp)[(NG + 1) / 2],
                                             const TC (*Dm)[NG / 2 > 0 ? NG / 2 : 1])
{
    constexpr int GE = NG / 2;
    TC vp[GE > 0 ? GE : 1], vm[GE > 0 ? GE : 1];
#pragma unroll
    for (int a = 0; a < GE; ++a) {
        vp[a] = v[a] + v[NG - 1 - a];
        vm[a] = v[a] - v[NG - 1 - a];
    }
#pragma unroll
    for (int m = 0; m < GE; ++m) {
        TC pp = 0, mm = 0;
#pragma unroll
        for (int a = 0; a < GE; ++a) pp += Dm[a][m] * vp[a];
        if constexpr (NG % 2 == 1) pp += Dm[GE][m] * v[GE];
#pragma unroll
        for (int a = 0; a < GE; ++a) mm += Dp[a][m] * vm[a];
        w[m] = mm + pp;
        w[NG - 1 - m] = mm - pp;
    }
    if constexpr (NG % 2 == 1) {
        TC mm = 0;
#pragma unroll
        for (int a = 0; a < GE; ++a) mm += Dp[a][GE] * vm[a];
        w[GE] = mm;
    }
}

// Half tables of the interpolation matrix I1d (FP64, Ng x Nq, row-major).
template <int NQ, class TC>
__device__ __forceinline__ void interp_half_tables(const double *__restrict__ I1d, TC (*Ie)[(NQ + 1) / 2],
                                                   TC (*Io)[NQ / 2 > 0 ? NQ / 2 : 1])
{
    constexpr int NG = NQ + 1, HG = (NG + 1) / 2, HQ = (NQ + 1) / 2, GE = NG / 2, QE = NQ / 2;
#pragma unroll
    for (int a = 0; a < HG; ++a)
#pragma unroll
        for (int m = 0; m < HQ; ++m) {
            const double v0 = I1d[a * NQ + m], v1 = I1d[a * NQ + NQ - 1 - m];
            Ie[a][m] = static_cast<TC>(m == NQ - 1 - m ? v0 : 0.5 * (v0 + v1));
            if (a < GE && m < QE) Io[a][m] = static_cast<TC>(0.5 * (v0 - v1));
        }
}

// Half tables of the Gauss-point derivative matrix Dgl (FP64, Ng x Ng).
template <int NG, class TC>
__device__ __forceinline__ void deriv_half_tables(const double *__restrict__ Dgl, TC (*Dp)[(NG + 1) / 2],
                                                  TC (*Dm)[NG / 2 > 0 ? NG / 2 : 1])
{
    constexpr int GE = NG / 2, HG = (NG + 1) / 2;
#pragma unroll
    for (int a = 0; a < HG; ++a)
#pragma unroll
        for (int m = 0; m < HG; ++m) {
            const double v0 = Dgl[a * NG + m], v1 = Dgl[a * NG + NG - 1 - m];
            if (a < GE) Dp[a][m] = static_cast<TC>(m == NG - 1 - m ? v0 : 0.5 * (v0 + v1));
            if (m < GE) Dm[a][m] = static_cast<TC>(0.5 * (v0 - v1));
        }
}

// The same half tables in LDS, for Nq beyond what the registers hold next to
// the lines.  Thread t of the workgroup fetches the pair of FP64 entries
// behind half-table entry t (the fetch goes out with the element's own loads
// and is waited for on its own), then stores the entry; the caller
// synchronises the workgroup before the tables are read.
template <int NQ>
__device__ __forceinline__ void interp_pair_load(const double *__restrict__ I1d, int t, double &v0, double &v1)
{
    constexpr int HG = (NQ + 2) / 2, HQ = (NQ + 1) / 2;
    const int tt = t < HG * HQ ? t : 0;
    const int a = tt / HQ, m = tt - a * HQ;
    v0 = I1d[a * NQ + m];
    v1 = I1d[a * NQ + NQ - 1 - m];
}

template <int NQ, class TC>
__device__ __forceinline__ void interp_pair_store(TC (*Ie)[(NQ + 1) / 2], TC (*Io)[NQ / 2 > 0 ? NQ / 2 : 1], int t,
                                                  double v0, double v1)
{
    constexpr int NG = NQ + 1, HG = (NG + 1) / 2, HQ = (NQ + 1) / 2, GE = NG / 2, QE = NQ / 2;
    if (t < HG * HQ) {
        const int a = t / HQ, m = t - a * HQ;
        Ie[a][m] = static_cast<TC>(m == NQ - 1 - m ? v0 : 0.5 * (v0 + v1));
        if (a < GE && m < QE) Io[a][m] = static_cast<TC>(0.5 * (v0 - v1));
    }
}

template <int NG>
__device__ __forceinline__ void deriv_pair_load(const double *__restrict__ Dgl, int t, double &v0, double &v1)
{
    constexpr int HG = (NG + 1) / 2;
    const int tt = t < HG * HG ? t : 0;
    const int a = tt / HG, m = tt - a * HG;
    v0 = Dgl[a * NG + m];
    v1 = Dgl[a * NG + NG - 1 - m];
}

template <int NG, class TC>
__device__ __forceinline__ void deriv_pair_store(TC (*Dp)[(NG + 1) / 2], TC (*Dm)[NG / 2 > 0 ? NG / 2 : 1], int t,
                                                 double v0, double v1)
{
    constexpr int GE = NG / 2, HG = (NG + 1) / 2;
    if (t < HG * HG) {
        const int a = t / HG, m = t - a * HG;
        if (a < GE) Dp[a][m] = static_cast<TC>(m == NG - 1 - m ? v0 : 0.5 * (v0 + v1));
        if (m < GE) Dm[a][m] = static_cast<TC>(0.5 * (v0 - v1));
    }
}

}  // namespace fem
