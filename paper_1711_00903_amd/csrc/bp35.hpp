// bp35.hpp -- BP3.5: collocated screened-Poisson operator on GLL nodes,
// y = (D^T G D + lambda J) u (Sec. "Benchmark Problem 3.5", Alg. 4).
//
// Thread layout: thread (i,j) of an element owns the column of nodes (i,j,k),
// k = 0..Nq-1, in registers (the z-sweep).  The t-derivative and its
// transpose never leave the registers; the r- and s-contractions read whole
// rows of a padded LDS volume.  Two workgroup barriers per element group:
// after u is staged, and after the weighted gradients (wr, ws) are staged.
#pragma once

#include "bp35t.hpp"
#include "fem_device.hpp"
#include "launch.hpp"
#include "tiles.hpp"

namespace fem {

// Vector of Nq table entries a thread uses in a contraction: either copied
// into registers once, or read from the LDS copy of the table on each use.
template <int LEN, bool REG, class TC>
struct TabVec {
    TC v[REG ? LEN : 1];
    const TC *p;
    int stride;
    __device__ __forceinline__ void init(const TC *lds, int base, int stride_)
    {
        if constexpr (REG) {
#pragma unroll
            for (int m = 0; m < LEN; ++m) v[m] = lds[base + m * stride_];
        } else {
            p = lds + base;
            stride = stride_;
        }
    }
    __device__ __forceinline__ TC operator[](int m) const
    {
        if constexpr (REG) return v[m];
        else return p[m * stride];
    }
};

// Table entry that is the same for every lane (index known at compile time):
// FP64 tables are read straight from global memory (scalar loads); reduced
// precision reads the LDS copy, which holds the converted values.
template <class TC>
__device__ __forceinline__ TC uniform_entry(const double *__restrict__ g, const TC *s, int idx)
{
    if constexpr (std::is_same<TC, double>::value) return g[idx];
    else return s[idx];
}

// The same, with the source chosen by the caller: SCALAR reads the FP64 table
// through the scalar cache, otherwise the LDS copy (broadcast reads).
template <bool SCALAR, class TC>
__device__ __forceinline__ TC table_entry(const double *__restrict__ g, const TC *s, int idx)
{
    if constexpr (SCALAR) return g[idx];
    else return s[idx];
}

// Stage the fields of a group of `nvalid` consecutive elements (contiguous in
// global memory) into LDS as [slot][k][j][i] with row length PQ.  Every thread
// issues all of its loads before its first LDS store, so the group's loads are
// in flight together instead of one round trip per loop iteration.
template <int NQ, int EPB, int NT, int SLOT, int PQ, class TC, class TV>
__device__ __forceinline__ void stage_fields(TC *__restrict__ s_w, const TV *__restrict__ ug, int nvalid)
{
    constexpr int NP = NQ * NQ * NQ;
    constexpr int NS = (EPB * NP + NT - 1) / NT;
    const int total = nvalid * NP;
    // unconditional loads (a clamped index past the group): a narrow value loaded
    // under a condition is widened inside the branch, one wait per load
    TV raw[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int x = static_cast<int>(threadIdx.x) + s * NT;
        raw[s] = ug[x < total ? x : 0];
    }
    TC v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = to_compute(raw[s], TC{});
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int x = static_cast<int>(threadIdx.x) + s * NT;
        if (x < total) {
            const int sl = x / NP, n = x - sl * NP;
            const int k = n / (NQ * NQ), r = n - k * NQ * NQ;
            const int jj = r / NQ, ii = r - jj * NQ;
            s_w[sl * SLOT + k * NQ * PQ + jj * PQ + ii] = v[s];
        }
    }
}

// XP: the conjugate-gradient direction update p <- r + beta_p p is applied to
// u in place as it is loaded (u is then read and written through `pw`, r is
// `xr`, beta_p is *xbeta), so the operator acts on the updated p.
template <int NQ, int EPB, class TG, class TV, bool XP = false>
__global__ __launch_bounds__(threads_for(1, NQ, EPB)) void bp35_kernel(
    int64_t E, int64_t ngroups, const double *__restrict__ D1d, const TG *__restrict__ G,
    const TG *__restrict__ wJ, typename compute_pair<TG, TV>::type lambda, const TV *__restrict__ u,
    typename output_of<TV>::type *__restrict__ y, typename compute_pair<TG, TV>::type beta,
    typename compute_pair<TG, TV>::type oscale, TV *pw = nullptr, const TV *__restrict__ xr = nullptr,
    const double *__restrict__ xbeta = nullptr, TV *__restrict__ xlo = nullptr,
    const double *__restrict__ xalpha = nullptr)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int P = lds_row(NQ, sizeof(TC));
    constexpr int SLAB = NQ * P;
    constexpr int VOL = NQ * SLAB;
    // Table rows in registers only for small Nq; for larger Nq the LDS copy
    // leaves the registers to the prefetched geometric factors.
    constexpr bool TREG = NQ <= 5;
    // All 6 Nq factors of a column are loaded before the first barrier, so the
    // element's whole HBM read is in flight at once; beyond Nq = 10 they no
    // longer fit in registers and each slab's factors are loaded as needed.
    constexpr bool PREF = NQ <= 10;
    constexpr int W = geo_vec(NQ, sizeof(TG));   // slabs per vector load of geometric data
    // Uniform table entries of the t-direction: with FP64 arithmetic on FP64
    // data through the scalar cache (the measured faster choice there); with
    // narrower geometric data the packed factors leave VGPRs free and the LDS
    // copy is faster than the SGPR spills the scalar entries cause.
    constexpr bool SCALAR_TAB = std::is_same<TC, double>::value && std::is_same<TG, double>::value;
    // 16-bit fields: the group's u block (contiguous) is fetched in 16-byte
    // pieces by all threads and staged in LDS, instead of Nq 2-byte loads per
    // lane (address-bound); each lane then reads its column back from LDS.
    constexpr int NT = threads_for(1, NQ, EPB);
    constexpr bool USTAGE = !XP && sizeof(TV) == 2 && (NP % 8) == 0;
    constexpr int UPIECES = EPB * NP / 8;
    constexpr int UPPT = (UPIECES + NT - 1) / NT;

    __shared__ TC s_D[NQ * NQ];
    __shared__ TC s_u[EPB * VOL];
    __shared__ TC s_r[EPB * VOL];
    __shared__ TC s_s[EPB * VOL];

    const int t = threadIdx.x;
    const int slot = t / NC;
    const int col = t - slot * NC;
    const int i = col % NQ;
    const int j = col / NQ;
    const bool lane = slot < EPB;
    const int sl = lane ? slot : 0;

    stage_table(s_D, D1d, NQ * NQ);
    __syncthreads();

    TabVec<NQ, TREG, TC> Di, Dj, DiT, DjT;   // D[i][m], D[j][m], D[m][i], D[m][j]
    Di.init(s_D, i * NQ, 1);
    Dj.init(s_D, j * NQ, 1);
    DiT.init(s_D, i, NQ);
    DjT.init(s_D, j, NQ);

    TC *su = s_u + sl * VOL;
    TC *sr = s_r + sl * VOL;
    TC *ss = s_s + sl * VOL;
    const int me = j * P + i;   // this column's offset inside a slab

    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int64_t e = g * EPB + slot;
        const bool ok = lane && e < E;
        const int64_t base = (ok ? e : 0) * NP + col;

        // Loads are issued by every lane (lanes without an element read element
        // 0 and never store): under a lane condition the compiler stops
        // counting the requests in flight and waits for the factors as well
        // before the field reaches LDS.
        TC uc[NQ];
        if constexpr (XP) {
            static_assert(std::is_same<TV, double>::value || std::is_same<TV, float>::value,
                          "direction update on FP64 or FP32 fields");
            const TC bp = static_cast<TC>(*xbeta);   // in the vectors' precision, as xpay_kernel
            // with xlo set, the previous step's iterate update x_lo += alpha p
            // is folded in here, on the p it read before replacing it
            const bool fold = xlo != nullptr;
            TV rv[NQ], xv[NQ];
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                uc[k] = pw[base + k * NC];
                rv[k] = xr[base + k * NC];
            }
            if (fold) {
#pragma unroll
                for (int k = 0; k < NQ; ++k) xv[k] = xlo[base + k * NC];
            }
            const TC al = fold ? static_cast<TC>(*xalpha) : TC(0);
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                if (fold) {
                    xv[k] += al * uc[k];
                    if (ok) xlo[base + k * NC] = xv[k];
                }
                uc[k] = rv[k] + bp * uc[k];
                if (ok) pw[base + k * NC] = uc[k];
            }
        } else if constexpr (!USTAGE) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = ld<TC>(u, base + k * NC);
        }
        using R16 = typename raw_vec<16>::type;
        R16 upc[USTAGE ? UPPT : 1];
        int npieces = 0;
        if constexpr (USTAGE) {
            const int64_t g0 = g * EPB;
            const int nvalid = static_cast<int>((E - g0) < EPB ? (E - g0) : EPB);
            npieces = nvalid * (NP / 8);
            const R16 *src = reinterpret_cast<const R16 *>(u + g0 * NP);
#pragma unroll
            for (int q = 0; q < UPPT; ++q) {
                const int t = static_cast<int>(threadIdx.x) + q * NT;
                upc[q] = t < npieces ? src[t] : R16{};
            }
        }
        const TG *Ge = G + (ok ? e : 0) * (6 * NP) + col * W;
        constexpr int NV = NQ / W;   // vectors per factor and column
        // gp[f * NV + k / W], lane k % W: factor f at slab k, stored precision
        packed_vec<W, TG> gp[PREF ? 6 * NV : 1];
        if constexpr (PREF) {
            // plain loads at Nq <= 3, where a slab of Nq^2 W values is a
            // fraction of a 128-byte line and non-temporal requests for the
            // slabs sharing a line fetched it from HBM once each
#pragma unroll
            for (int f = 0; f < 6; ++f)
#pragma unroll
                for (int kq = 0; kq < NV; ++kq) {
                    if constexpr (NQ <= 3) gp[f * NV + kq].load(Ge + f * NP + kq * NC * W);
                    else gp[f * NV + kq].stream(Ge + f * NP + kq * NC * W);
                }
        }
        // beyond Nq = 10 the factors of each group of W slabs are requested
        // GDIST groups ahead of their use (occupancy is one wave per SIMD
        // there, so the wave's own requests must cover the HBM latency).
        // Measured at E = 262144: +4..23% for Nq = 11..14; at Nq >= 15 the
        // extra registers cost more than the latency they hide, so the factors
        // are requested at use.
        constexpr int GDIST = NQ >= 15 ? 0 : 2;
        packed_vec<W, TG> gq[PREF ? 1 : NV][6];
        if constexpr (!PREF) {
#pragma unroll
            for (int q = 0; q < (GDIST < NV ? GDIST : NV); ++q)
#pragma unroll
                for (int f = 0; f < 6; ++f) gq[q][f].stream(Ge + f * NP + q * NC * W);
        }
        if constexpr (USTAGE) {
#pragma unroll
            for (int q = 0; q < UPPT; ++q) {
                const int t = static_cast<int>(threadIdx.x) + q * NT;
                if (t < npieces) {
                    TV tmp[8];
                    __builtin_memcpy(tmp, &upc[q], 16);
#pragma unroll
                    for (int v = 0; v < 8; ++v) {
                        const int n0 = t * 8 + v;
                        const int gs = n0 / NP, n = n0 - gs * NP;
                        const int k = n / NC, r = n - k * NC;
                        const int jj = r / NQ, ii = r - jj * NQ;
                        s_u[gs * VOL + k * SLAB + jj * P + ii] = to_compute(tmp[v], TC{});
                    }
                }
            }
        } else if (lane) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) su[k * SLAB + me] = uc[k];
        }
        __syncthreads();
        if constexpr (USTAGE) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = su[k * SLAB + me];
        }

        TC wt[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            TC qr = 0, qs = 0, qt = 0;
            const TC *row = su + k * SLAB + j * P;   // u[k][j][*]
            const TC *cln = su + k * SLAB + i;       // u[k][*][i]
#pragma unroll
            for (int m = 0; m < NQ; ++m) {
                qr += Di[m] * row[m];
                qs += Dj[m] * cln[m * P];
                qt += table_entry<SCALAR_TAB>(D1d, s_D, k * NQ + m) * uc[m];
            }
            TC grr = 0, grs = 0, grt = 0, gss = 0, gst = 0, gtt = 0;
            if constexpr (PREF) {
                grr = gp[0 * NV + k / W].template get<TC>(k % W);
                grs = gp[1 * NV + k / W].template get<TC>(k % W);
                grt = gp[2 * NV + k / W].template get<TC>(k % W);
                gss = gp[3 * NV + k / W].template get<TC>(k % W);
                gst = gp[4 * NV + k / W].template get<TC>(k % W);
                gtt = gp[5 * NV + k / W].template get<TC>(k % W);
            } else if (ok) {
                if (k % W == 0 && k / W + GDIST < NV) {
#pragma unroll
                    for (int f = 0; f < 6; ++f) gq[k / W + GDIST][f].stream(Ge + f * NP + (k / W + GDIST) * NC * W);
                }
                grr = gq[k / W][0].template get<TC>(k % W);
                grs = gq[k / W][1].template get<TC>(k % W);
                grt = gq[k / W][2].template get<TC>(k % W);
                gss = gq[k / W][3].template get<TC>(k % W);
                gst = gq[k / W][4].template get<TC>(k % W);
                gtt = gq[k / W][5].template get<TC>(k % W);
            }
            const TC wr = grr * qr + grs * qs + grt * qt;
            const TC ws = grs * qr + gss * qs + gst * qt;
            wt[k] = grt * qr + gst * qs + gtt * qt;
            if (lane) {
                sr[k * SLAB + me] = wr;
                ss[k * SLAB + me] = ws;
            }
        }
        __syncthreads();

#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            TC acc = 0;
            const TC *rrow = sr + k * SLAB + j * P;   // wr[k][j][*]
            const TC *scol = ss + k * SLAB + i;       // ws[k][*][i]
#pragma unroll
            for (int m = 0; m < NQ; ++m) {
                acc += DiT[m] * rrow[m];
                acc += DjT[m] * scol[m * P];
                acc += table_entry<SCALAR_TAB>(D1d, s_D, m * NQ + k) * wt[m];
            }
            if (ok) {
                const int64_t idx = base + k * NC;
                if (lambda != TC(0))
                    acc += lambda * ld<TC>(wJ, (ok ? e : 0) * NP + geo_offset(col, k, NQ, W)) * uc[k];
                acc *= oscale;
                if (beta != TC(0)) acc += beta * static_cast<TC>(y[idx]);
                y[idx] = static_cast<TY>(acc);
            }
        }
        // No third barrier: the next group writes s_u only after all lanes have
        // passed the barrier above (so every read of s_u is done), and writes
        // s_r / s_s only after its own first barrier, which every lane reaches
        // after finishing the reads of this group.
    }
}

template <int NQ, int EPB, class TG, class TV>
hipError_t bp35_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    const int64_t ngroups = (a.E + EPB - 1) / EPB;
    int64_t grid = ngroups;
    if (a.grid_cap > 0 && grid > a.grid_cap) grid = a.grid_cap;
    if (grid > max_grid(threads_for(1, NQ, EPB))) grid = max_grid(threads_for(1, NQ, EPB));
    if (grid < 1) return hipSuccess;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    // the direction update: FP64 fields at every degree the CG split serves,
    // FP32 fields (the iterative-refinement inner CG) likewise
    if constexpr (std::is_same<TV, double>::value || (std::is_same<TV, float>::value && NQ <= 8)) {
        if (a.xr) {
            hipLaunchKernelGGL((bp35_kernel<NQ, EPB, TG, TV, true>), dim3(static_cast<unsigned>(grid)),
                               dim3(threads_for(1, NQ, EPB)), 0, s, a.E, ngroups, a.D1d,
                               static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                               static_cast<TC>(a.lambda), static_cast<const TV *>(a.u),
                               static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale,
                               static_cast<TV *>(const_cast<void *>(a.u)), static_cast<const TV *>(a.xr),
                               a.xbeta, static_cast<TV *>(a.xl), a.xalpha);
            return hipGetLastError();
        }
    }
    if (a.xr) return hipErrorInvalidValue;
    hipLaunchKernelGGL((bp35_kernel<NQ, EPB, TG, TV>), dim3(static_cast<unsigned>(grid)),
                       dim3(threads_for(1, NQ, EPB)), 0, s, a.E, ngroups, a.D1d,
                       static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                       static_cast<TC>(a.lambda), static_cast<const TV *>(a.u),
                       static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale);
    return hipGetLastError();
}

template <int NQ, class TG, class TV>
hipError_t bp35_launch_nq(const ApplyArgs &a, hipStream_t s)
{
    constexpr auto ch = epb_choices(1, NQ);
    const int epb = a.epb > 0 ? a.epb : epb_default(1, NQ);
    // one element per workgroup at high degree: the line-per-lane kernel (the
    // direction update of the conjugate-gradient split stays on the column kernel)
    if constexpr (bp35_line(NQ, 1)) {
        if (epb == 1 && !a.xr) return bp35t_launch_t<NQ, TG, TV>(a, s);
    }
    if (epb == ch[0]) return bp35_launch_t<NQ, ch[0], TG, TV>(a, s);
    if constexpr (ch[1] > 0) if (epb == ch[1]) return bp35_launch_t<NQ, ch[1], TG, TV>(a, s);
    if constexpr (ch[2] > 0) if (epb == ch[2]) return bp35_launch_t<NQ, ch[2], TG, TV>(a, s);
    if constexpr (ch[3] > 0) if (epb == ch[3]) return bp35_launch_t<NQ, ch[3], TG, TV>(a, s);
    return hipErrorInvalidConfiguration;
}

template <class TG, class TV>
hipError_t bp35_launch(const ApplyArgs &a, hipStream_t s)
{
    switch (a.N + 1) {
    case 2: return bp35_launch_nq<2, TG, TV>(a, s);
    case 3: return bp35_launch_nq<3, TG, TV>(a, s);
    case 4: return bp35_launch_nq<4, TG, TV>(a, s);
    case 5: return bp35_launch_nq<5, TG, TV>(a, s);
    case 6: return bp35_launch_nq<6, TG, TV>(a, s);
    case 7: return bp35_launch_nq<7, TG, TV>(a, s);
    case 8: return bp35_launch_nq<8, TG, TV>(a, s);
    case 9: return bp35_launch_nq<9, TG, TV>(a, s);
    case 10: return bp35_launch_nq<10, TG, TV>(a, s);
    case 11: return bp35_launch_nq<11, TG, TV>(a, s);
    case 12: return bp35_launch_nq<12, TG, TV>(a, s);
    case 13: return bp35_launch_nq<13, TG, TV>(a, s);
    case 14: return bp35_launch_nq<14, TG, TV>(a, s);
    case 15: return bp35_launch_nq<15, TG, TV>(a, s);
    case 16: return bp35_launch_nq<16, TG, TV>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
