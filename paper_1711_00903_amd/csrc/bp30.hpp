// bp30.hpp -- BP3.0: de-aliased screened-Poisson operator
// y = I^T (D~^T G D~ + lambda J) I u on the (N+2)^3 Gauss grid (Sec. "BP3.0",
// Alg. 5, with interpolation / projection of Alg. 1-2).
//
// Thread layout: one thread per (a,b) column of the Ng x Ng Gauss grid.  The
// field interpolated to the Gauss grid, q~[c] (c = 0..Ng-1), stays in the
// thread's registers from the t-interpolation through the t-derivative and the
// lambda term; the t-contractions of the stiffness and of the projection are
// register-local as well.  LDS holds the r/s slabs:
//   R1: u[k][j][i]  -> q~[c][b][a] -> V[k][b][a]
//   R2: T[k][j][a]  -> wr[c][b][a] -> W[k][j][a]
//   R3: ws[c][b][a]
// Six workgroup barriers per element group.
#pragma once

#include "bp35.hpp"
#include "bp30t.hpp"

namespace fem {

// Minimum waves per SIMD asked of the register allocator.  At Nq = 8 the
// multi-element packings then fit 256 VGPRs without spills and run two waves
// per SIMD instead of one (4.0 instead of 5.7 ms at N = 7, E = 262144);
// elsewhere the cap would spill, so it is not set.  (One element per
// workgroup runs bp30t_kernel instead.)
constexpr int bp30_min_waves(int nq, int epb) { return (nq == 8 && epb > 1) ? 2 : 1; }

template <int NQ, int EPB, class TG, class TV>
__global__ __launch_bounds__(threads_for(2, NQ, EPB))
__attribute__((amdgpu_waves_per_eu(bp30_min_waves(NQ, EPB)))) void bp30_kernel(
    int64_t E, int64_t ngroups, const double *__restrict__ I1d, const double *__restrict__ Dgl,
    const TG *__restrict__ G, const TG *__restrict__ wJ, typename compute_pair<TG, TV>::type lambda,
    const TV *__restrict__ u, typename output_of<TV>::type *__restrict__ y,
    typename compute_pair<TG, TV>::type beta, typename compute_pair<TG, TV>::type oscale)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NG = NQ + 1;
    constexpr int NP = NQ * NQ * NQ;
    constexpr int NPG = NG * NG * NG;
    constexpr int NCG = NG * NG;
    constexpr int PQ = lds_row(NQ, sizeof(TC));
    constexpr int PG = lds_row(NG, sizeof(TC));
    constexpr int R1a = NQ * NQ * PQ, R1b = NG * NG * PG, R1c = NQ * NG * PG;
    constexpr int R1 = R1a > R1b ? (R1a > R1c ? R1a : R1c) : (R1b > R1c ? R1b : R1c);
    constexpr int R2a = NQ * NQ * PG, R2b = NG * NG * PG;
    constexpr int R2 = R2a > R2b ? R2a : R2b;
    constexpr int SLOT = bp30_slot_values(NQ, sizeof(TC));
    static_assert(SLOT == R1 + R2 + NG * NG * PG, "LDS slot layout");
    constexpr bool TREG = NQ <= 6;
    constexpr int W = geo_vec(NG, sizeof(TG));   // Gauss slabs per vector load of G / wJ

    __shared__ TC s_I[NG * NQ];
    __shared__ TC s_D[NG * NG];
    __shared__ TC s_w[EPB * SLOT];

    const int t = threadIdx.x;
    const int slot = t / NCG;
    const int col = t - slot * NCG;
    const bool lane = slot < EPB;
    const int sl = lane ? slot : 0;
    const int a = col % NG, b = col / NG;
    const int i4 = col % NQ, j4 = col / NQ;
    const bool ph13 = lane && b < NQ;
    const bool ph4 = lane && col < NQ * NQ;

    stage_table(s_I, I1d, NG * NQ);
    stage_table(s_D, Dgl, NG * NG);
    __syncthreads();

    TabVec<NQ, TREG, TC> Ia, Ib;      // I[a][*], I[b][*]
    TabVec<NG, TREG, TC> Icj, Ici;    // I[*][b] (b < NQ), I[*][i4]
    TabVec<NG, TREG, TC> Da, Db, DaT, DbT;   // D~[a][*], D~[b][*], D~[*][a], D~[*][b]
    Ia.init(s_I, a * NQ, 1);
    Ib.init(s_I, b * NQ, 1);
    Icj.init(s_I, b < NQ ? b : 0, NQ);
    Ici.init(s_I, i4, NQ);
    Da.init(s_D, a * NG, 1);
    Db.init(s_D, b * NG, 1);
    DaT.init(s_D, a, NG);
    DbT.init(s_D, b, NG);

    TC *r1 = s_w + sl * SLOT;
    TC *r2 = r1 + R1;
    TC *r3 = r2 + R2;
    const int meg = b * PG + a;   // (a,b) inside a Gauss slab

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t e0 = g * EPB;
        {
            const int nvalid = static_cast<int>((E - e0) < EPB ? (E - e0) : EPB);
            stage_fields<NQ, EPB, threads_for(2, NQ, EPB), SLOT, PQ>(s_w, u + e0 * NP, nvalid);
        }
        const int64_t e = e0 + slot;
        const bool ok = lane && e < E;
        const TG *Ge = G + (ok ? e : 0) * (6 * NPG) + col * W;
        // Ng <= 5: all of the column's factors are requested here, together
        // with u, and kept in their stored type until the metric step; loaded
        // there, slab by slab, each request was waited for in turn after the
        // interpolations (one exposed round trip per W slabs at low degree).
        // Plain loads: a slab of Ng^2 W values is a fraction of a 128-byte
        // line, and non-temporal requests for the slabs sharing a line fetched
        // it from HBM once each (1.95x the algorithmic bytes at N = 1).  FP64
        // factors at Ng = 4 stay on the slab path (8% slower prefetched).
        constexpr bool GPREF = NG <= 3 || (NG <= 5 && sizeof(TG) < 8);
        constexpr int NVG = NG / W;
        packed_vec<W, TG> gpv[GPREF ? 6 * NVG : 1];
        if constexpr (GPREF) {
#pragma unroll
            for (int f = 0; f < 6; ++f)
#pragma unroll
                for (int cq = 0; cq < NVG; ++cq) gpv[f * NVG + cq].load(Ge + f * NPG + cq * NCG * W);
        }
        __syncthreads();

        // r-interpolation: T[k][j][a] = sum_i I[a][i] u[k][j][i]   (R1 -> R2)
        if (ph13) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = r1 + k * NQ * PQ + b * PQ;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Ia[m] * row[m];
                r2[k * NQ * PG + b * PG + a] = s;
            }
        }
        __syncthreads();

        // s- and t-interpolation into registers: q~[c] at Gauss node (a,b,c)
        TC qg[NG];
        {
            TC T2[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = r2 + k * NQ * PG + a;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Ib[m] * cl[m * PG];
                T2[k] = s;
            }
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                TC s = 0;
#pragma unroll
                for (int k = 0; k < NQ; ++k) s += uniform_entry(I1d, s_I, c * NQ + k) * T2[k];
                qg[c] = s;
            }
        }
        if (lane) {
#pragma unroll
            for (int c = 0; c < NG; ++c) r1[c * NG * PG + meg] = qg[c];
        }
        __syncthreads();

        // gradient on the Gauss grid, metric, weighted gradient (R1 -> R2, R3)
        TC wt[NG];
        TC gw[6 * W];   // the six factors of W Gauss slabs
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            const TC *row = r1 + c * NG * PG + b * PG;   // q~[c][b][*]
            const TC *cl = r1 + c * NG * PG + a;          // q~[c][*][a]
            TC qr = 0, qs = 0, qt = 0;
#pragma unroll
            for (int m = 0; m < NG; ++m) {
                qr += Da[m] * row[m];
                qs += Db[m] * cl[m * PG];
                qt += uniform_entry(Dgl, s_D, c * NG + m) * qg[m];
            }
            TC grr = 0, grs = 0, grt = 0, gss = 0, gst = 0, gtt = 0;
            if constexpr (GPREF) {
                if (ok) {
                    grr = gpv[0 * NVG + c / W].template get<TC>(c % W);
                    grs = gpv[1 * NVG + c / W].template get<TC>(c % W);
                    grt = gpv[2 * NVG + c / W].template get<TC>(c % W);
                    gss = gpv[3 * NVG + c / W].template get<TC>(c % W);
                    gst = gpv[4 * NVG + c / W].template get<TC>(c % W);
                    gtt = gpv[5 * NVG + c / W].template get<TC>(c % W);
                }
            } else if (ok) {
                if (c % W == 0) {
#pragma unroll
                    for (int f = 0; f < 6; ++f) ld_stream_vec<W>(Ge + f * NPG + (c / W) * NCG * W, gw + f * W);
                }
                grr = gw[0 * W + c % W];
                grs = gw[1 * W + c % W];
                grt = gw[2 * W + c % W];
                gss = gw[3 * W + c % W];
                gst = gw[4 * W + c % W];
                gtt = gw[5 * W + c % W];
            }
            if (lane) {
                r2[c * NG * PG + meg] = grr * qr + grs * qs + grt * qt;
                r3[c * NG * PG + meg] = grs * qr + gss * qs + gst * qt;
            }
            wt[c] = grt * qr + gst * qs + gtt * qt;
        }
        __syncthreads();

        // transposed gradient, lambda term, t-projection into registers
        TC V[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) V[k] = 0;
        const TG *wJe = wJ + (ok ? e : 0) * NPG + col * W;
        TC wjv[W];
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            const TC *rrow = r2 + c * NG * PG + b * PG;   // wr[c][b][*]
            const TC *scol = r3 + c * NG * PG + a;        // ws[c][*][a]
            TC s = 0;
#pragma unroll
            for (int m = 0; m < NG; ++m) {
                s += DaT[m] * rrow[m];
                s += DbT[m] * scol[m * PG];
                s += uniform_entry(Dgl, s_D, m * NG + c) * wt[m];
            }
            if (lambda != TC(0) && ok) {
                if (c % W == 0) ld_stream_vec<W>(wJe + (c / W) * NCG * W, wjv);
                s += lambda * wjv[c % W] * qg[c];
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) V[k] += uniform_entry(I1d, s_I, c * NQ + k) * s;
        }
        // R1 (q~) was last read before the previous barrier: V can overwrite it.
        if (lane) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) r1[k * NG * PG + meg] = V[k];
        }
        __syncthreads();

        // s-projection: W[k][j][a] = sum_b I[b][j] V[k][b][a]   (R1 -> R2)
        if (ph13) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = r1 + k * NG * PG + a;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NG; ++m) s += Icj[m] * cl[m * PG];
                r2[k * NQ * PG + b * PG + a] = s;
            }
        }
        __syncthreads();

        // r-projection: y[k][j][i] = sum_a I[a][i] W[k][j][a]
        if (ph4 && ok) {
            const int64_t base = e * NP + j4 * NQ + i4;
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = r2 + k * NQ * PG + j4 * PG;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NG; ++m) s += Ici[m] * row[m];
                s *= oscale;
                const int64_t idx = base + k * NQ * NQ;
                if (beta != TC(0)) s += beta * static_cast<TC>(y[idx]);
                y[idx] = static_cast<TY>(s);
            }
        }
        // The next group writes R1 (staging) after this point: R1 was last
        // read in the s-projection, two barriers ago.  R2 is rewritten only
        // after the next staging barrier, which follows this r-projection.
    }
}

template <int NQ, int EPB, class TG, class TV>
hipError_t bp30_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    const int64_t ngroups = (a.E + EPB - 1) / EPB;
    int64_t grid = ngroups;
    if (a.grid_cap > 0 && grid > a.grid_cap) grid = a.grid_cap;
    if (grid > max_grid(threads_for(2, NQ, EPB))) grid = max_grid(threads_for(2, NQ, EPB));
    if (grid < 1) return hipSuccess;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    hipLaunchKernelGGL((bp30_kernel<NQ, EPB, TG, TV>), dim3(static_cast<unsigned>(grid)),
                       dim3(threads_for(2, NQ, EPB)), 0, s, a.E, ngroups, a.I1d, a.Dgl,
                       static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                       static_cast<TC>(a.lambda), static_cast<const TV *>(a.u),
                       static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale);
    return hipGetLastError();
}

template <int NQ, class TG, class TV>
hipError_t bp30_launch_nq(const ApplyArgs &a, hipStream_t s)
{
    constexpr auto ch = epb_choices(2, NQ);
    const int epb = a.epb > 0 ? a.epb : epb_default(2, NQ);
    if (epb == ch[0]) {
        if constexpr (bp30_line(NQ, ch[0])) return bp30t_launch_t<NQ, TG, TV>(a, s);
        else return bp30_launch_t<NQ, ch[0], TG, TV>(a, s);
    }
    if constexpr (ch[1] > 0) if (epb == ch[1]) return bp30_launch_t<NQ, ch[1], TG, TV>(a, s);
    if constexpr (ch[2] > 0) if (epb == ch[2]) return bp30_launch_t<NQ, ch[2], TG, TV>(a, s);
    if constexpr (ch[3] > 0) if (epb == ch[3]) return bp30_launch_t<NQ, ch[3], TG, TV>(a, s);
    return hipErrorInvalidConfiguration;
}

template <class TG, class TV>
hipError_t bp30_launch(const ApplyArgs &a, hipStream_t s)
{
    switch (a.N + 1) {
    case 2: return bp30_launch_nq<2, TG, TV>(a, s);
    case 3: return bp30_launch_nq<3, TG, TV>(a, s);
    case 4: return bp30_launch_nq<4, TG, TV>(a, s);
    case 5: return bp30_launch_nq<5, TG, TV>(a, s);
    case 6: return bp30_launch_nq<6, TG, TV>(a, s);
    case 7: return bp30_launch_nq<7, TG, TV>(a, s);
    case 8: return bp30_launch_nq<8, TG, TV>(a, s);
    case 9: return bp30_launch_nq<9, TG, TV>(a, s);
    case 10: return bp30_launch_nq<10, TG, TV>(a, s);
    case 11: return bp30_launch_nq<11, TG, TV>(a, s);
    case 12: return bp30_launch_nq<12, TG, TV>(a, s);
    case 13: return bp30_launch_nq<13, TG, TV>(a, s);
    case 14: return bp30_launch_nq<14, TG, TV>(a, s);
    case 15: return bp30_launch_nq<15, TG, TV>(a, s);
    case 16: return bp30_launch_nq<16, TG, TV>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
