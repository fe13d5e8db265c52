// bp10.hpp -- BP1.0: mass operator y = I^T J I u (Sec. "Benchmark Problem 1",
// Alg. 1-3).
//
// Thread layout: one thread per (a,b) column of the Ng x Ng Gauss grid of an
// element.  The six one-direction contractions run as
//   r-interpolation      LDS u[k][j][*]   -> LDS T[k][j][a]      threads (a,j)
//   s-interpolation      LDS T[k][*][a]   -> registers T2[k]     threads (a,b)
//   t-interpolation, scaling by wJ, t-projection, all in registers (a,b)
//   s-projection         LDS V[k][*][a]   -> LDS W[k][j][a]      threads (a,j)
//   r-projection         LDS W[k][j][*]   -> global y[k][j][i]   threads (i,j)
// with four workgroup barriers per element group (after staging u, after each
// LDS-to-LDS phase).  The t-direction never touches LDS, so each Gauss column
// is interpolated, scaled and projected back inside one thread.
#pragma once

#include "bp35.hpp"
#include "bp10t.hpp"
#include "bp10tp.hpp"

namespace fem {

template <int NQ, int EPB, class TG, class TV>
__global__ __launch_bounds__(threads_for(0, NQ, EPB)) void bp10_kernel(
    int64_t E, int64_t ngroups, const double *__restrict__ I1d, const TG *__restrict__ wJ,
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
    constexpr int SU = NQ * NQ * PQ;   // u[k][j][i]
    constexpr int SA = NQ * NQ * PG;   // T[k][j][a] and W[k][j][a]
    constexpr int SB = NQ * NG * PG;   // V[k][b][a]
    constexpr int SLOT = SU + SA + SB;
    constexpr bool TREG = NQ <= 8;
    constexpr int W = geo_vec(NG, sizeof(TG));   // Gauss slabs per vector load of wJ

    __shared__ TC s_I[NG * NQ];
    __shared__ TC s_w[EPB * SLOT];

    const int t = threadIdx.x;
    const int slot = t / NCG;
    const int col = t - slot * NCG;
    const bool lane = slot < EPB;
    const int sl = lane ? slot : 0;
    // (a,b) on the Gauss grid; the same thread is (a,jj) with jj = b in the
    // half-projected phases and (i,j) in the GLL phase.
    const int a = col % NG, b = col / NG;
    const int i4 = col % NQ, j4 = col / NQ;
    const bool ph13 = lane && b < NQ;          // (a, j) threads
    const bool ph4 = lane && col < NQ * NQ;    // (i, j) threads

    stage_table(s_I, I1d, NG * NQ);
    __syncthreads();

    TabVec<NQ, TREG, TC> Ia, Ib;    // I[a][*], I[b][*]
    TabVec<NG, TREG, TC> Icj, Ici;  // I[*][b] (b as the GLL index j), I[*][i4]
    Ia.init(s_I, a * NQ, 1);
    Ib.init(s_I, (b < NG ? b : 0) * NQ, 1);
    Icj.init(s_I, b < NQ ? b : 0, NQ);
    Ici.init(s_I, i4, NQ);

    TC *su = s_w + sl * SLOT;
    TC *sa = su + SU;
    TC *sb = sa + SA;

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t e0 = g * EPB;
        // stage u of the group's elements (contiguous in global memory)
        {
            const int nvalid = static_cast<int>((E - e0) < EPB ? (E - e0) : EPB);
            stage_fields<NQ, EPB, threads_for(0, NQ, EPB), SLOT, PQ>(s_w, u + e0 * NP, nvalid);
        }
        const int64_t e = e0 + slot;
        const bool ok = lane && e < E;
        // The element's scaled Jacobians (this Gauss column) and, with beta, the
        // old output are requested now, so their latency overlaps the
        // interpolation phases.
        TC wj[NG];
        if (ok) {
            const TG *wJe = wJ + e * NPG + col * W;
            if constexpr (NG <= 4 || (NG == 5 && sizeof(TG) < 8)) {
                // plain loads at low degree: a slab of Ng^2 W values is a
                // fraction of a 128-byte line, and non-temporal requests for
                // the slabs sharing a line fetched it from HBM once each
                // (FP64 at Ng = 5 measured 7% slower with them)
#pragma unroll
                for (int cq = 0; cq < NG / W; ++cq) ld_vec<W>(wJe + cq * NCG * W, wj + cq * W);
            } else {
#pragma unroll
                for (int cq = 0; cq < NG / W; ++cq) ld_stream_vec<W>(wJe + cq * NCG * W, wj + cq * W);
            }
        } else {
#pragma unroll
            for (int c = 0; c < NG; ++c) wj[c] = TC(0);
        }
        TC yold[NQ];
        if (beta != TC(0) && ph4 && ok) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) yold[k] = static_cast<TC>(y[e * NP + j4 * NQ + i4 + k * NQ * NQ]);
        }
        __syncthreads();

        // r-interpolation: T[k][j][a] = sum_i I[a][i] u[k][j][i]
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
        __syncthreads();

        // s-interpolation into registers, then the whole t-direction.
        TC V[NQ];
        {
            TC T2[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = sa + k * NQ * PG + a;   // T[k][*][a]
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NQ; ++m) s += Ib[m] * cl[m * PG];
                T2[k] = s;
            }
#pragma unroll
            for (int k = 0; k < NQ; ++k) V[k] = 0;
#pragma unroll
            for (int c = 0; c < NG; ++c) {
                TC q = 0;
#pragma unroll
                for (int k = 0; k < NQ; ++k) q += uniform_entry(I1d, s_I, c * NQ + k) * T2[k];
                const TC wq = q * wj[c];
#pragma unroll
                for (int k = 0; k < NQ; ++k) V[k] += uniform_entry(I1d, s_I, c * NQ + k) * wq;
            }
        }
        if (lane) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) sb[k * NG * PG + b * PG + a] = V[k];
        }
        __syncthreads();

        // s-projection: W[k][j][a] = sum_b I[b][j] V[k][b][a]
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
        __syncthreads();

        // r-projection: y[k][j][i] = sum_a I[a][i] W[k][j][a]
        if (ph4 && ok) {
            const int64_t base = e * NP + j4 * NQ + i4;
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = sa + k * NQ * PG + j4 * PG;
                TC s = 0;
#pragma unroll
                for (int m = 0; m < NG; ++m) s += Ici[m] * row[m];
                s *= oscale;
                const int64_t idx = base + k * NQ * NQ;
                if (beta != TC(0)) s += beta * yold[k];
                y[idx] = static_cast<TY>(s);
            }
        }
        // The next group stages u only into s_u (read in the r-interpolation of
        // this group, which all lanes finished two barriers ago) and then
        // passes a barrier before sa is rewritten, so no barrier is needed here.
    }
}

template <int NQ, int EPB, class TG, class TV>
hipError_t bp10_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    if (a.part) return hipErrorInvalidValue;   // element partials: one-wave kernel only
    const int64_t ngroups = (a.E + EPB - 1) / EPB;
    int64_t grid = ngroups;
    if (a.grid_cap > 0 && grid > a.grid_cap) grid = a.grid_cap;
    if (grid > max_grid(threads_for(0, NQ, EPB))) grid = max_grid(threads_for(0, NQ, EPB));
    if (grid < 1) return hipSuccess;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    hipLaunchKernelGGL((bp10_kernel<NQ, EPB, TG, TV>), dim3(static_cast<unsigned>(grid)),
                       dim3(threads_for(0, NQ, EPB)), 0, s, a.E, ngroups, a.I1d,
                       static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u),
                       static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale);
    return hipGetLastError();
}

template <int NQ, class TG, class TV>
hipError_t bp10_launch_nq(const ApplyArgs &a, hipStream_t s)
{
    constexpr auto ch = epb_choices(0, NQ);
    const int epb = a.epb > 0 ? a.epb : epb_default(0, NQ);
    if (epb == ch[0]) {
        if constexpr (bp10_wave(NQ, ch[0])) {
            if constexpr (bp10tp_use(NQ, static_cast<int>(sizeof(TG)), static_cast<int>(sizeof(TV))))
                return bp10tp_launch_t<NQ, TG, TV>(a, s);
            return bp10t_launch_t<NQ, TG, TV>(a, s);
        }
        else return bp10_launch_t<NQ, ch[0], TG, TV>(a, s);
    }
    if constexpr (ch[1] > 0) if (epb == ch[1]) return bp10_launch_t<NQ, ch[1], TG, TV>(a, s);
    if constexpr (ch[2] > 0) if (epb == ch[2]) return bp10_launch_t<NQ, ch[2], TG, TV>(a, s);
    if constexpr (ch[3] > 0) if (epb == ch[3]) return bp10_launch_t<NQ, ch[3], TG, TV>(a, s);
    return hipErrorInvalidConfiguration;
}

template <class TG, class TV>
hipError_t bp10_launch(const ApplyArgs &a, hipStream_t s)
{
    switch (a.N + 1) {
    case 2: return bp10_launch_nq<2, TG, TV>(a, s);
    case 3: return bp10_launch_nq<3, TG, TV>(a, s);
    case 4: return bp10_launch_nq<4, TG, TV>(a, s);
    case 5: return bp10_launch_nq<5, TG, TV>(a, s);
    case 6: return bp10_launch_nq<6, TG, TV>(a, s);
    case 7: return bp10_launch_nq<7, TG, TV>(a, s);
    case 8: return bp10_launch_nq<8, TG, TV>(a, s);
    case 9: return bp10_launch_nq<9, TG, TV>(a, s);
    case 10: return bp10_launch_nq<10, TG, TV>(a, s);
    case 11: return bp10_launch_nq<11, TG, TV>(a, s);
    case 12: return bp10_launch_nq<12, TG, TV>(a, s);
    case 13: return bp10_launch_nq<13, TG, TV>(a, s);
    case 14: return bp10_launch_nq<14, TG, TV>(a, s);
    case 15: return bp10_launch_nq<15, TG, TV>(a, s);
    case 16: return bp10_launch_nq<16, TG, TV>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
