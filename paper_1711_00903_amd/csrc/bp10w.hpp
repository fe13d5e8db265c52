// bp10w.hpp -- BP1.0 mass operator with one wave64 per element (Nq^2 <= 64,
// i.e. N <= 7), using the centro-symmetry of the interpolation matrix.
//
// The same six one-direction contractions as bp10.hpp (Alg. 1-3), but:
//   * every phase of an element runs inside one wave, so the workgroup
//     barriers synchronise a single wave;
//   * each 1-D contraction uses I[a][i] = I[Ng-1-a][Nq-1-i] (the symmetry the
//     BP1.0 optimisation section exploits in its Kernel 8), in even-odd form:
//     with x+ = x_i + x_{n-1-i}, x- = x_i - x_{n-1-i} and the half tables
//         Ie[a][i] = (I[a][i] + I[a][n-1-i]) / 2,  Io[a][i] = (I[a][i] - I[a][n-1-i]) / 2,
//     one lane reads the n inputs once and produces both outputs,
//         y_a = e + o,  y_{m-1-a} = e - o,  e = sum Ie x+ (+ I[a][mid] x_mid),  o = sum Io x-,
//     which halves the LDS reads and the FLOPs of the contractions.
// The projections (I^T) have the same symmetry.  Phases, with the lanes each
// uses (Ng = Nq + 1 Gauss points, h = ceil(Ng/2), q = Nq/2):
//   r-interpolation  u[k][j][*] -> T[k][j][a], T[k][j][Ng-1-a]   lanes (a<h, j)
//   s-interpolation  T[k][*][a] -> columns (a,b), (a,Ng-1-b)      lanes (a, b<h)
//     + t-interpolation, x wJ, t-projection in registers, -> V[k][b][a]
//   s-projection     V[k][*][a] -> W[k][j][a], W[k][Nq-1-j][a]   lanes (a, j<q)
//   r-projection     W[k][j][*] -> y[k][j][i], y[k][j][Nq-1-i]   lanes (i<q, j)
#pragma once

#include "bp35.hpp"

namespace fem {

// DOT: also write part[e] = sum over the element's nodes of u * y (y the final
// output), reduced across the wave in a fixed order.
template <int NQ, class TG, class TV, bool DOT = false>
__global__ __launch_bounds__(kWave) void bp10w_kernel(
    int64_t E, const double *__restrict__ I1d, const TG *__restrict__ wJ, const TV *__restrict__ u,
    typename output_of<TV>::type *__restrict__ y, typename compute_pair<TG, TV>::type beta,
    typename compute_pair<TG, TV>::type oscale, double *__restrict__ part = nullptr, int64_t e0 = 0)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NG = NQ + 1;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int NCG = NG * NG;
    constexpr int NPG = NCG * NG;
    constexpr int HG = (NG + 1) / 2;   // Gauss index pairs (with the middle one when Ng is odd)
    constexpr int HQ = (NQ + 1) / 2;   // GLL index pairs
    constexpr int QE = NQ / 2;         // full GLL pairs
    constexpr int GE = NG / 2;         // full Gauss pairs
    constexpr int PQ = lds_row(NQ, sizeof(TC));
    constexpr int PG = lds_row(NG, sizeof(TC));
    constexpr int W = geo_vec(NG, sizeof(TG));
    static_assert(NC <= kWave && HG * NQ <= kWave && NG * HG <= kWave, "one wave per element");

    // Interpolation, even-odd: rows a < HG, columns i < HQ (Ie includes the middle column).
    __shared__ TC s_ie[HG * HQ];
    __shared__ TC s_io[HG * HQ];
    // Projection (I^T: Nq x Ng), even-odd: rows j < HQ, columns b < HG.
    __shared__ TC s_pe[HQ * HG];
    __shared__ TC s_po[HQ * HG];
    // the full table in the compute precision for uniform reads (an FP64
    // kernel reads those from global memory through the scalar cache)
    constexpr bool SI = !std::is_same<TC, double>::value;
    __shared__ TC s_I[SI ? NG * NQ : 1];
    // u[k][j][i] is dead once the r-interpolation has read it, so V[k][b][a]
    // reuses its space
    constexpr int SU = NQ * NQ * PQ, SB = NQ * NG * PG;
    __shared__ TC sub[SU > SB ? SU : SB];
    __shared__ TC sa[NQ * NQ * PG];   // T[k][j][a], then W[k][j][a]
    TC *const su = sub, *const sb = sub;
    // Scaled Jacobians narrower than FP64: the element's Ng^3 contiguous values
    // are fetched as whole dwords by every lane (coalesced) and staged in LDS,
    // instead of 2 Ng strided 2- or 4-byte loads per lane.  The dwords
    // [d0, d1) are those wholly inside the element's block plus, for 16-bit
    // values with an odd first index, the half-filled first one; a last value
    // that shares its dword with the next element is fetched on its own.
    constexpr bool WST = sizeof(TG) < 8;
    constexpr int VPD = WST ? 4 / static_cast<int>(sizeof(TG)) : 1;   // values per dword
    constexpr int NDW = WST ? NPG / VPD + 1 : 1;
    constexpr int DPL = (NDW + kWave - 1) / kWave;                     // dword loads per lane
    __shared__ uint32_t s_wd[NDW];

    const int L = threadIdx.x;
    if constexpr (SI) stage_table(s_I, I1d, NG * NQ);
    // half tables from the FP64 interpolation matrix I1d[a][i] (Ng x Nq)
    for (int x = L; x < HG * HQ; x += kWave) {
        const int a = x / HQ, i = x % HQ;
        const double v0 = I1d[a * NQ + i], v1 = I1d[a * NQ + NQ - 1 - i];
        s_ie[x] = static_cast<TC>(i == NQ - 1 - i ? v0 : 0.5 * (v0 + v1));
        s_io[x] = static_cast<TC>(0.5 * (v0 - v1));
    }
    for (int x = L; x < HQ * HG; x += kWave) {
        const int j = x / HG, b = x % HG;   // I^T[j][b] = I[b][j]
        const double v0 = I1d[b * NQ + j], v1 = I1d[(NG - 1 - b) * NQ + j];
        s_pe[x] = static_cast<TC>(b == NG - 1 - b ? v0 : 0.5 * (v0 + v1));
        s_po[x] = static_cast<TC>(0.5 * (v0 - v1));
    }

    const bool gll = L < NC;
    const bool p2 = L < NG * HG;
    const int a2 = L % NG, b2 = L / NG;               // s-interpolation lane: column (a2, b2), (a2, Ng-1-b2)
    const bool two = p2 && (b2 != NG - 1 - b2);
    const int c0 = a2 + NG * b2, c1 = a2 + NG * (NG - 1 - b2);
    // requests of element e: the u column of (i,j) = (L % Nq, L / Nq) and the
    // wJ of the two Gauss columns of this lane's s-interpolation
    auto request = [&](int64_t e, TC *uc, TC *wj0, TC *wj1) {
        const int64_t base = e * NP + (gll ? L : 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k) uc[k] = gll ? ld<TC>(u, base + k * NC) : TC(0);
        if constexpr (!WST) {
            const TG *wJe = wJ + e * NPG;
#pragma unroll
            for (int cq = 0; cq < NG / W; ++cq) {
                if (p2) ld_stream_vec<W>(wJe + c0 * W + cq * NCG * W, wj0 + cq * W);
                if (two) ld_stream_vec<W>(wJe + c1 * W + cq * NCG * W, wj1 + cq * W);
            }
        }
    };
    // One element per workgroup, no loop: a loop over elements would keep the
    // loop-invariant table rows of all four phases in registers.
    {
        const int64_t e = e0 + blockIdx.x;
        TC uc[NQ], wj0[NG], wj1[NG];
        request(e, uc, wj0, wj1);
        const int64_t v0 = e * NPG;                     // first wJ value of the element
        const int64_t d0 = v0 / VPD, nd = (v0 + NPG) / VPD - d0;
        const int off = static_cast<int>(v0 - d0 * VPD);   // its index inside the staged dwords
        uint32_t wst[WST ? DPL : 1];
        uint16_t wlast = 0;
        const bool tail = WST && VPD == 2 && ((v0 + NPG) % 2) == 1;
        if constexpr (WST) {
            const uint32_t *wd = reinterpret_cast<const uint32_t *>(wJ) + d0;
#pragma unroll
            for (int q = 0; q < DPL; ++q) {
                const int t = L + q * kWave;
                wst[q] = t < nd ? __builtin_nontemporal_load(wd + t) : 0u;
            }
            if (tail && L == 0) wlast = reinterpret_cast<const uint16_t *>(wJ)[v0 + NPG - 1];
        }
        if (gll) {
            const int i = L % NQ, j = L / NQ;
#pragma unroll
            for (int k = 0; k < NQ; ++k) su[k * NQ * PQ + j * PQ + i] = uc[k];
        }
        __syncthreads();

        // r-interpolation: lanes (a < HG, j)
        if (L < HG * NQ) {
            const int a = L % HG, jj = L / HG;
            TC ie[HQ], io[QE > 0 ? QE : 1];
#pragma unroll
            for (int m = 0; m < HQ; ++m) ie[m] = s_ie[a * HQ + m];
#pragma unroll
            for (int m = 0; m < QE; ++m) io[m] = s_io[a * HQ + m];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = su + k * NQ * PQ + jj * PQ;
                TC x[NQ];
#pragma unroll
                for (int m = 0; m < NQ; ++m) x[m] = row[m];
                TC ev = 0, od = 0;
#pragma unroll
                for (int m = 0; m < QE; ++m) {
                    ev += ie[m] * (x[m] + x[NQ - 1 - m]);
                    od += io[m] * (x[m] - x[NQ - 1 - m]);
                }
                if constexpr (NQ % 2 == 1) ev += ie[QE] * x[QE];
                sa[k * NQ * PG + jj * PG + a] = ev + od;
                if (a != NG - 1 - a) sa[k * NQ * PG + jj * PG + NG - 1 - a] = ev - od;
            }
        }
        if constexpr (WST) {
#pragma unroll
            for (int q = 0; q < DPL; ++q) {
                const int t = L + q * kWave;
                if (t < nd) s_wd[t] = wst[q];
            }
            if (tail && L == 0) reinterpret_cast<uint16_t *>(s_wd)[off + NPG - 1] = wlast;
        }
        __syncthreads();

        // s-interpolation of columns (a2, b2) and (a2, Ng-1-b2), then the t-direction of each
        if (p2) {
            if constexpr (WST) {
                const TG *sw = reinterpret_cast<const TG *>(s_wd) + off;
#pragma unroll
                for (int c = 0; c < NG; ++c) {
                    wj0[c] = to_compute(sw[c0 + c * NCG], TC{});
                    wj1[c] = two ? to_compute(sw[c1 + c * NCG], TC{}) : TC(0);
                }
            }
            TC Tp[NQ], Tm[NQ];
            {
                TC ie[HQ], io[QE > 0 ? QE : 1];
#pragma unroll
                for (int m = 0; m < HQ; ++m) ie[m] = s_ie[b2 * HQ + m];
#pragma unroll
                for (int m = 0; m < QE; ++m) io[m] = s_io[b2 * HQ + m];
#pragma unroll
                for (int k = 0; k < NQ; ++k) {
                    const TC *cl = sa + k * NQ * PG + a2;   // T[k][*][a2]
                    TC x[NQ];
#pragma unroll
                    for (int m = 0; m < NQ; ++m) x[m] = cl[m * PG];
                    TC ev = 0, od = 0;
#pragma unroll
                    for (int m = 0; m < QE; ++m) {
                        ev += ie[m] * (x[m] + x[NQ - 1 - m]);
                        od += io[m] * (x[m] - x[NQ - 1 - m]);
                    }
                    if constexpr (NQ % 2 == 1) ev += ie[QE] * x[QE];
                    Tp[k] = ev + od;   // column b2
                    Tm[k] = ev - od;   // column Ng-1-b2
                }
            }
            // t-direction of one column: V[k] = sum_c I[c][k] wJ[c] sum_k' I[c][k'] T[k']
            auto tdir = [&](const TC *T, const TC *wj, TC *V) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) V[k] = 0;
#pragma unroll
                for (int c = 0; c < NG; ++c) {
                    TC q = 0;
#pragma unroll
                    for (int k = 0; k < NQ; ++k) q += uniform_entry(I1d, s_I, c * NQ + k) * T[k];
                    const TC wq = q * wj[c];
#pragma unroll
                    for (int k = 0; k < NQ; ++k) V[k] += uniform_entry(I1d, s_I, c * NQ + k) * wq;
                }
            };
            TC V[NQ];
            tdir(Tp, wj0, V);
#pragma unroll
            for (int k = 0; k < NQ; ++k) sb[k * NG * PG + b2 * PG + a2] = V[k];
            if (two) {
                tdir(Tm, wj1, V);
#pragma unroll
                for (int k = 0; k < NQ; ++k) sb[k * NG * PG + (NG - 1 - b2) * PG + a2] = V[k];
            }
        }
        __syncthreads();

        // s-projection: lanes (a, j < HQ): W[k][j][a], W[k][Nq-1-j][a] from V[k][*][a]
        if (L < NG * HQ) {
            const int a = L % NG, jj = L / NG;
            TC pe[HG], po[GE > 0 ? GE : 1];
#pragma unroll
            for (int m = 0; m < HG; ++m) pe[m] = s_pe[jj * HG + m];
#pragma unroll
            for (int m = 0; m < GE; ++m) po[m] = s_po[jj * HG + m];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *cl = sb + k * NG * PG + a;
                TC x[NG];
#pragma unroll
                for (int m = 0; m < NG; ++m) x[m] = cl[m * PG];
                TC ev = 0, od = 0;
#pragma unroll
                for (int m = 0; m < GE; ++m) {
                    ev += pe[m] * (x[m] + x[NG - 1 - m]);
                    od += po[m] * (x[m] - x[NG - 1 - m]);
                }
                if constexpr (NG % 2 == 1) ev += pe[GE] * x[GE];
                sa[k * NQ * PG + jj * PG + a] = ev + od;
                if (jj != NQ - 1 - jj) sa[k * NQ * PG + (NQ - 1 - jj) * PG + a] = ev - od;
            }
        }
        __syncthreads();

        // r-projection: lanes (i < HQ, j): y[k][j][i], y[k][j][Nq-1-i] from W[k][j][*]
        double dp = 0.0;
        if (L < HQ * NQ) {
            const int ii = L % HQ, jj = L / HQ;
            TC pe[HG], po[GE > 0 ? GE : 1];
#pragma unroll
            for (int m = 0; m < HG; ++m) pe[m] = s_pe[ii * HG + m];
#pragma unroll
            for (int m = 0; m < GE; ++m) po[m] = s_po[ii * HG + m];
            const int64_t yb = e * NP + jj * NQ;
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                const TC *row = sa + k * NQ * PG + jj * PG;
                TC x[NG];
#pragma unroll
                for (int m = 0; m < NG; ++m) x[m] = row[m];
                TC ev = 0, od = 0;
#pragma unroll
                for (int m = 0; m < GE; ++m) {
                    ev += pe[m] * (x[m] + x[NG - 1 - m]);
                    od += po[m] * (x[m] - x[NG - 1 - m]);
                }
                if constexpr (NG % 2 == 1) ev += pe[GE] * x[GE];
                TC y0 = (ev + od) * oscale, y1 = (ev - od) * oscale;
                const int64_t i0 = yb + k * NC + ii, i1 = yb + k * NC + (NQ - 1 - ii);
                if (beta != TC(0)) {
                    y0 += beta * static_cast<TC>(y[i0]);
                    y1 += beta * static_cast<TC>(y[i1]);
                }
                y[i0] = static_cast<TY>(y0);
                if (ii != NQ - 1 - ii) y[i1] = static_cast<TY>(y1);
                if constexpr (DOT) {
                    dp += u[i0] * y0;
                    if (ii != NQ - 1 - ii) dp += u[i1] * y1;
                }
            }
        }
        if constexpr (DOT) {
            static_assert(std::is_same<TV, double>::value, "element partials of FP64 fields");
#pragma unroll
            for (int off = kWave / 2; off > 0; off >>= 1) dp += __shfl_xor(dp, off);
            if (L == 0) part[e] = dp;
        }
    }
}

template <int NQ, class TG, class TV>
hipError_t bp10w_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    if (a.E < 1) return hipSuccess;
    if (a.part && !std::is_same<TV, double>::value) return hipErrorInvalidValue;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    // one workgroup per element; a grid cap splits the elements over launches
    const int64_t chunk = a.grid_cap > 0 ? a.grid_cap : a.E;
    for (int64_t e0 = 0; e0 < a.E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(a.E - e0 < chunk ? a.E - e0 : chunk);
        if constexpr (std::is_same<TV, double>::value) {
            if (a.part) {
                hipLaunchKernelGGL((bp10w_kernel<NQ, TG, TV, true>), dim3(grid), dim3(kWave), 0, s, a.E, a.I1d,
                                   static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u),
                                   static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale, a.part, e0);
                continue;
            }
        }
        hipLaunchKernelGGL((bp10w_kernel<NQ, TG, TV>), dim3(grid), dim3(kWave), 0, s, a.E, a.I1d,
                           static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u),
                           static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale, nullptr, e0);
    }
    return hipGetLastError();
}

}  // namespace fem
