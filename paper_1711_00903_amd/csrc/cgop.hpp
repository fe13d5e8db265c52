// cgop.hpp -- the CG operator in one pass: for each element,
//     p  <- r + beta p                       (optional; the CG direction update)
//     Ap <- S p + lambda M p                 (BP3.5 stiffness + BP1.0 mass)
//     partial sum of p . Ap for this workgroup
// with S the GLL-collocated stiffness (Alg. 4) and M the GL mass (Alg. 1-3).
//
// Thread layout: one thread per (a,b) column of the Ng x Ng Gauss grid, as in
// the BP1.0 kernel; the first Nq^2 threads of an element also own the (i,j)
// GLL columns of the stiffness, as in the BP3.5 kernel.  The field p is
// loaded once (per GLL column, into registers and the LDS volume) and feeds
// both operators; all geometric data of the element is requested before the
// first barrier.  Four workgroup barriers per element group:
//   1. p staged            -> stiffness gradients | mass r-interpolation
//   2. wr, ws, T staged    -> stiffness transposes | mass s/t-interpolation, scaling, t-projection
//   3. V staged            -> mass s-projection
//   4. W staged            -> mass r-projection, Ap = S p + lambda M p, store, p . Ap
#pragma once

#include "bp35.hpp"

namespace fem {

constexpr int cgop_slot_values(int nq, int bytes)
{
    const int ng = nq + 1;
    const int pq = lds_row(nq, bytes), pg = lds_row(ng, bytes);
    // u, wr, ws on the GLL grid; T / W [k][j][a]; V [k][b][a]
    return 3 * nq * nq * pq + nq * nq * pg + nq * ng * pg;
}

constexpr int cgop_epb(int nq)
{
    const int cols = (nq + 1) * (nq + 1);
    int epb = 256 / cols;
    if (epb < 1) epb = 1;
    while (epb > 1 && cgop_slot_values(nq, 8) * 8 * epb > 80 * 1024) --epb;
    return epb;
}

// The one-pass kernel fits the LDS of a workgroup up to Nq = 15 (N = 14);
// beyond that the CG uses the separate operator kernels.
constexpr bool cgop_fits(int nq)
{
    return (cgop_slot_values(nq, 8) * cgop_epb(nq) + nq * nq + (nq + 1) * nq + 8) * 8 <= kMaxLds;
}

template <int NQ, int EPB, class TG>
__global__ __launch_bounds__(threads_for(0, NQ, EPB)) void cgop_kernel(
    int64_t E, const double *__restrict__ I1d, const double *__restrict__ D1d,
    const TG *__restrict__ G, const TG *__restrict__ wJ, double s_scale, double m_scale,
    const double *__restrict__ r, double *__restrict__ p, const double *__restrict__ beta_ptr,
    int do_xpay, double *__restrict__ Ap, double *__restrict__ part)
{
    using TC = double;
    constexpr int NG = NQ + 1;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int NCG = NG * NG;
    constexpr int NPG = NCG * NG;
    constexpr int NT = threads_for(0, NQ, EPB);
    constexpr int PQ = lds_row(NQ, 8);
    constexpr int PG = lds_row(NG, 8);
    constexpr int SU = NQ * NQ * PQ;
    constexpr int SA = NQ * NQ * PG;
    constexpr int SLOT = cgop_slot_values(NQ, 8);
    constexpr int WS = geo_vec(NQ, sizeof(TG));   // GLL data interleave
    constexpr int WM = geo_vec(NG, sizeof(TG));   // GL data interleave

    __shared__ TC s_D[NQ * NQ];
    __shared__ TC s_I[NG * NQ];
    __shared__ TC s_w[EPB * SLOT];
    __shared__ double s_red[NT / kWave];

    const int t = threadIdx.x;
    const int slot = t / NCG;
    const int col = t - slot * NCG;
    const bool lane = slot < EPB;
    const int sl = lane ? slot : 0;
    const int a = col % NG, b = col / NG;          // Gauss column (a,b); also (a,j) with j = b
    const int i = col % NQ, j = col / NQ;          // GLL column (i,j) for col < Nq^2
    const bool gll = lane && col < NC;
    const bool ph13 = lane && b < NQ;

    stage_table(s_D, D1d, NQ * NQ);
    stage_table(s_I, I1d, NG * NQ);
    __syncthreads();

    TabVec<NQ, false, TC> Di, Dj, DiT, DjT;
    Di.init(s_D, (gll ? i : 0) * NQ, 1);
    Dj.init(s_D, (gll ? j : 0) * NQ, 1);
    DiT.init(s_D, gll ? i : 0, NQ);
    DjT.init(s_D, gll ? j : 0, NQ);
    TabVec<NQ, false, TC> Ia, Ib;
    TabVec<NG, false, TC> Icj, Ici;
    Ia.init(s_I, a * NQ, 1);
    Ib.init(s_I, b * NQ, 1);
    Icj.init(s_I, b < NQ ? b : 0, NQ);
    Ici.init(s_I, gll ? i : 0, NQ);

    TC *su = s_w + sl * SLOT;
    TC *sr = su + SU;
    TC *ss = sr + SU;
    TC *sa = ss + SU;
    TC *sb = sa + SA;
    const int me = j * PQ + i;

    const TC beta = do_xpay ? *beta_ptr : 0.0;
    const int64_t ngroups = (E + EPB - 1) / EPB;
    double acc_dot = 0.0;

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t e = g * EPB + slot;
        const bool ok = lane && e < E;
        const bool okc = ok && col < NC;
        const int64_t base = (ok ? e : 0) * NP + (gll ? j * NQ + i : 0);

        // p (with the direction update) for this GLL column
        TC uc[NQ];
        if (okc) {
            // p and r requested together before the update (with the update
            // inside the same loop, each r load was waited for right away)
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = p[base + k * NC];
            if (do_xpay) {
                TC rv[NQ];
#pragma unroll
                for (int k = 0; k < NQ; ++k) rv[k] = r[base + k * NC];
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    uc[k] = rv[k] + beta * uc[k];
                    p[base + k * NC] = uc[k];
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = 0.0;
        }
        // all geometric data of the element
        TC gp[6 * NQ];
        if (okc) {
            const TG *Ge = G + e * (6 * NP) + col * WS;
#pragma unroll
            for (int f = 0; f < 6; ++f)
#pragma unroll
                for (int kq = 0; kq < NQ / WS; ++kq)
                    ld_stream_vec<WS>(Ge + f * NP + kq * NC * WS, gp + f * NQ + kq * WS);
        } else {
#pragma unroll
            for (int x = 0; x < 6 * NQ; ++x) gp[x] = 0.0;
        }
        TC wj[NG];
        if (ok) {
            const TG *wJe = wJ + e * NPG + col * WM;
#pragma unroll
            for (int cq = 0; cq < NG / WM; ++cq) ld_stream_vec<WM>(wJe + cq * NCG * WM, wj + cq * WM);
        } else {
#pragma unroll
            for (int c = 0; c < NG; ++c) wj[c] = 0.0;
        }
        if (gll) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) su[k * NQ * PQ + me] = uc[k];
        }
        __syncthreads();   // 1

        // stiffness: gradients, metric, weighted gradients
        TC wt[NQ];
        if (gll) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = su + k * NQ * PQ + j * PQ;
                const TC *cln = su + k * NQ * PQ + i;
                TC qr = 0, qs = 0, qt = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    qr += Di[m] * row[m];
                    qs += Dj[m] * cln[m * PQ];
                    qt += D1d[k * NQ + m] * uc[m];
                }
                const TC grr = gp[0 * NQ + k], grs = gp[1 * NQ + k], grt = gp[2 * NQ + k];
                const TC gss = gp[3 * NQ + k], gst = gp[4 * NQ + k], gtt = gp[5 * NQ + k];
                sr[k * NQ * PQ + me] = grr * qr + grs * qs + grt * qt;
                ss[k * NQ * PQ + me] = grs * qr + gss * qs + gst * qt;
                wt[k] = grt * qr + gst * qs + gtt * qt;
            }
        }
        // mass: r-interpolation T[k][j][a] = sum_i I[a][i] p[k][j][i]
        if (ph13) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = su + k * NQ * PQ + b * PQ;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Ia[m] * row[m];
                sa[k * NQ * PG + b * PG + a] = s;
            }
        }
        __syncthreads();   // 2

        // stiffness transposes (registers)
        TC ys[NQ];
        if (gll) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *rrow = sr + k * NQ * PQ + j * PQ;
                const TC *scol = ss + k * NQ * PQ + i;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) {
                    s += DiT[m] * rrow[m];
                    s += DjT[m] * scol[m * PQ];
                    s += D1d[m * NQ + k] * wt[m];
                }
                ys[k] = s;
            }
        }
        // mass: s-interpolation, t-interpolation, scaling, t-projection
        {
            TC T2[NQ], V[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = sa + k * NQ * PG + a;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Ib[m] * cl[m * PG];
                T2[k] = s;
                V[k] = 0;
            }
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                TC q = 0;
#pragma unroll
                for (int k = 0; k < NQ; ++k) q += I1d[c * NQ + k] * T2[k];
                const TC wq = q * wj[c];
#pragma unroll
                for (int k = 0; k < NQ; ++k) V[k] += I1d[c * NQ + k] * wq;
            }
            if (lane) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) sb[k * NG * PG + b * PG + a] = V[k];
            }
        }
        __syncthreads();   // 3

        // mass: s-projection W[k][j][a] = sum_b I[b][j] V[k][b][a] (T is dead)
        if (ph13) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = sb + k * NG * PG + a;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NG; ++m) s += Icj[m] * cl[m * PG];
                sa[k * NQ * PG + b * PG + a] = s;
            }
        }
        __syncthreads();   // 4

        // mass: r-projection; combine, store, p . Ap
        if (okc) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = sa + k * NQ * PG + j * PG;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NG; ++m) s += Ici[m] * row[m];
                const TC y = s_scale * ys[k] + m_scale * s;
                Ap[base + k * NC] = y;
                acc_dot += y * uc[k];
            }
        }
        // The next group writes su after this point: su was last read in the
        // phases before barrier 2.  sr/ss/sa/sb are rewritten only after the
        // next group's barrier 1, which follows every read below barrier 4.
    }

    // workgroup partial of p . Ap (fixed order: lanes, then waves)
    double v = acc_dot;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    if ((t & (kWave - 1)) == 0) s_red[t / kWave] = v;
    __syncthreads();
    if (t == 0) {
        double s = 0;
#pragma unroll
        for (int w = 0; w < NT / kWave; ++w) s += s_red[w];
        part[blockIdx.x] = s;
    }
}

struct CgopArgs {
    int N;
    int64_t E;
    const double *I1d, *D1d;
    const void *G, *wJ;
    double s_scale, m_scale;      // Ap = s_scale S p + m_scale M p
    const double *r;
    double *p;
    const double *beta;           // device scalar
    int do_xpay;
    double *Ap;
    double *part;                 // one partial of p . Ap per workgroup
};

// Workgroups of one CG-operator launch (one per element group).
inline int64_t cgop_groups(int N, int64_t E)
{
    constexpr int epb[kMaxN + 2] = {1, 1, cgop_epb(2), cgop_epb(3), cgop_epb(4), cgop_epb(5), cgop_epb(6),
                                    cgop_epb(7), cgop_epb(8), cgop_epb(9), cgop_epb(10), cgop_epb(11),
                                    cgop_epb(12), cgop_epb(13), cgop_epb(14), cgop_epb(15), cgop_epb(16)};
    constexpr int threads[kMaxN + 2] = {64, 64, threads_for(0, 2, cgop_epb(2)), threads_for(0, 3, cgop_epb(3)),
                                        threads_for(0, 4, cgop_epb(4)), threads_for(0, 5, cgop_epb(5)),
                                        threads_for(0, 6, cgop_epb(6)), threads_for(0, 7, cgop_epb(7)),
                                        threads_for(0, 8, cgop_epb(8)), threads_for(0, 9, cgop_epb(9)),
                                        threads_for(0, 10, cgop_epb(10)), threads_for(0, 11, cgop_epb(11)),
                                        threads_for(0, 12, cgop_epb(12)), threads_for(0, 13, cgop_epb(13)),
                                        threads_for(0, 14, cgop_epb(14)), threads_for(0, 15, cgop_epb(15)),
                                        threads_for(0, 16, cgop_epb(16))};
    const int e = epb[N + 1];
    const int64_t g = (E + e - 1) / e;
    return g < max_grid(threads[N + 1]) ? g : max_grid(threads[N + 1]);
}

template <int NQ, class TG>
hipError_t cgop_launch_nq(const CgopArgs &a, hipStream_t s)
{
    static_assert(cgop_fits(NQ), "one-pass CG operator exceeds the LDS of a workgroup");
    constexpr int EPB = cgop_epb(NQ);
    // the kernel loops over element groups beyond the grid; the partial count
    // (cgop_groups) is the grid
    int64_t grid = (a.E + EPB - 1) / EPB;
    if (grid > max_grid(threads_for(0, NQ, EPB))) grid = max_grid(threads_for(0, NQ, EPB));
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL((cgop_kernel<NQ, EPB, TG>), dim3(static_cast<unsigned>(grid)),
                       dim3(threads_for(0, NQ, EPB)), 0, s, a.E, a.I1d, a.D1d,
                       static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ), a.s_scale,
                       a.m_scale, a.r, a.p, a.beta, a.do_xpay, a.Ap, a.part);
    return hipGetLastError();
}

template <class TG>
hipError_t cgop_launch(const CgopArgs &a, hipStream_t s)
{
    switch (a.N + 1) {
    case 2: return cgop_launch_nq<2, TG>(a, s);
    case 3: return cgop_launch_nq<3, TG>(a, s);
    case 4: return cgop_launch_nq<4, TG>(a, s);
    case 5: return cgop_launch_nq<5, TG>(a, s);
    case 6: return cgop_launch_nq<6, TG>(a, s);
    case 7: return cgop_launch_nq<7, TG>(a, s);
    case 8: return cgop_launch_nq<8, TG>(a, s);
    case 9: return cgop_launch_nq<9, TG>(a, s);
    case 10: return cgop_launch_nq<10, TG>(a, s);
    case 11: return cgop_launch_nq<11, TG>(a, s);
    case 12: return cgop_launch_nq<12, TG>(a, s);
    case 13: return cgop_launch_nq<13, TG>(a, s);
    case 14: return cgop_launch_nq<14, TG>(a, s);
    case 15: return cgop_launch_nq<15, TG>(a, s);
    default: return hipErrorInvalidValue;   // Nq = 16 does not fit: see cgop_fits
    }
}

inline bool cgop_supported(int N)
{
    switch (N + 1) {
    case 2: return cgop_fits(2);
    case 3: return cgop_fits(3);
    case 4: return cgop_fits(4);
    case 5: return cgop_fits(5);
    case 6: return cgop_fits(6);
    case 7: return cgop_fits(7);
    case 8: return cgop_fits(8);
    case 9: return cgop_fits(9);
    case 10: return cgop_fits(10);
    case 11: return cgop_fits(11);
    case 12: return cgop_fits(12);
    case 13: return cgop_fits(13);
    case 14: return cgop_fits(14);
    case 15: return cgop_fits(15);
    default: return false;
    }
}

}  // namespace fem
