// bp10t.hpp -- BP1.0 mass operator, one element per workgroup of
// ceil(Nq^2 / 64) waves, with every one-direction contraction done by a lane
// that owns a whole line.
//
// The six contractions of Alg. 1-3 (interpolate t, s, r; scale by wJ; project
// r, s, t) are each a small matrix times one line of the element.  Here a lane
// holds the line in registers and produces all outputs of that line with the
// uniform 1-D table, and the element is turned between line directions
// through LDS (one write and one read per point), instead of every lane
// reading a whole LDS line for each single output.  Each line product uses
// the centro-symmetry I[a][i] = I[Ng-1-a][Nq-1-i] (the symmetry the BP1.0
// optimisation section exploits) in even-odd form: with the half tables
//     Ie[a][m] = (I[a][m] + I[a][Nq-1-m]) / 2   (a < ceil(Ng/2), m < ceil(Nq/2))
//     Io[a][m] = (I[a][m] - I[a][Nq-1-m]) / 2   (a < floor(Ng/2), m < floor(Nq/2))
// interpolation of a line x (Nq values) to Gauss points is
//     y_a = e_a + o_a,  y_{Ng-1-a} = e_a - o_a,
//     e_a = sum_m Ie[a][m] (x_m + x_{Nq-1-m}) [+ Ie[a][mid] x_mid],  o_a = sum_m Io[a][m] (x_m - x_{Nq-1-m}),
// and projection (I^T) of a Gauss line v uses the same half tables with the
// roles of the indices exchanged.
//
// Phases (N = 7: Nq = 8, Ng = 9, one wave; a phase with more lines than the
// workgroup has lanes takes a second pass over the first lanes):
//   t-interpolation  lanes (i,j): u column in registers -> A[c][j][i]          64 lines
//   s-interpolation  lines (i,c): A[c][*][i]            -> B[c][b][i]          72 lines
//   r-direction      lines (b,c): B[c][b][*] -> interpolate, x wJ, project -> B[c][b][*] (in place)   81 lines
//   s-projection     lines (i,c): B[c][*][i]            -> A[c][j][i]          72 lines
//   t-projection     lanes (i,j): A[*][j][i]            -> y[k][j][i]          64 lines
// The element's scaled Jacobians (one contiguous block) are fetched by every
// lane in coalesced pieces at the start and staged in A once the
// s-interpolation has consumed it.
#pragma once

#include "bp35.hpp"
#include "lines.hpp"

namespace fem {

// DOT: also write part[e] = sum over the element's nodes of u * y (y the final
// output), reduced across the wave in a fixed order.
constexpr int bp10t_threads(int nq) { return round_up_wave(nq * nq); }

template <int NQ, class TG, class TV, bool DOT = false>
__global__ __launch_bounds__(bp10t_threads(NQ)) void bp10t_kernel(
    int64_t E, const double *__restrict__ I1d, const TG *__restrict__ wJ, const TV *__restrict__ u,
    typename output_of<TV>::type *__restrict__ y, typename compute_pair<TG, TV>::type beta,
    typename compute_pair<TG, TV>::type oscale, double *__restrict__ part = nullptr, int64_t e0 = 0)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NG = NQ + 1;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int NPG = NG * NG * NG;
    constexpr int HG = (NG + 1) / 2, HQ = (NQ + 1) / 2, GE = NG / 2, QE = NQ / 2;
    // row length of both LDS volumes (rows along i); FP64 at Nq = 16 takes odd
    // rows (17, not the 18 of the bank model), which brings the workgroup's
    // LDS under 80 KB, so two of them share a CU (2.1 -> 3.0 TB/s at E = 65536)
    constexpr int P = bp10t_row(NQ, sizeof(TC));
    constexpr int SA = NQ * P;                   // slab of A: [j][i]
    constexpr int SB = NG * P;                   // slab of B: [b][i]
    constexpr int W = geo_vec(NG, sizeof(TG));   // interleave of the geometric layout
    constexpr int NT = bp10t_threads(NQ);
    static_assert(NC <= NT, "one lane per GLL column");

    // A: t-interpolated field [c][j][i], then the staged wJ, then the
    // s-projected field [c][j][i].  B: s-interpolated field [c][b][i], turned
    // in place into the r-direction result [c][b][i].  The staged wJ keeps its
    // stored type.  Where Ng W (the interleave) times the value size is a
    // multiple of 256 bytes (Ng = 16), the lanes of an r-direction pass,
    // reading it in its global layout, all fall on one bank (an LDS conflict
    // ratio of 0.72 for BF16 at N = 14): there it is staged in rows [c][b][a]
    // of odd length PW (6-8% faster).  Elsewhere the remap costs more than the
    // conflicts (5-20% slower) and the pieces are copied as they are.
    constexpr bool REMAP = bp10t_remap_w(NG, static_cast<int>(sizeof(TG)));
    constexpr int PW = bp10t_wrow(NG);
    constexpr int WBYTES = REMAP ? NG * NG * PW * static_cast<int>(sizeof(TG))
                                 : NPG * static_cast<int>(sizeof(TG)) + 8;   // (+ misalignment slack)
    constexpr int AV = NG * SA;
    constexpr int A_VALUES = AV * static_cast<int>(sizeof(TC)) > WBYTES ? AV
                                                                        : (WBYTES + sizeof(TC) - 1) / sizeof(TC);
    __shared__ __align__(16) TC sA[A_VALUES];
    __shared__ __align__(16) TC sB[NG * SB];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;

    // half tables, uniform across the wave: in registers for small Nq, in LDS
    // from Nq = 12 (the lines then need the registers); the LDS copy is
    // fetched before the element's loads and stored after they are issued.
    constexpr bool TLDS = NQ >= 12;
    // FP64 from Nq = 11: an empty asm with a memory clobber between line
    // products that share a table (the r-direction's interpolation and
    // projection; from Nq = 12 also the lines of the s-direction) makes each
    // read the table again instead of the compiler holding the first one's
    // values in registers for the next (measured at E = 65536: Nq = 11 3.3 ->
    // 3.9, Nq = 12 3.2 -> 3.7 (with the tables in LDS), Nq = 13 2.8 -> 3.1,
    // Nq = 14 2.5 -> 3.0, Nq = 15 2.4 -> 3.0 TB/s).  In FP32 arithmetic the
    // same fences cut the registers (Nq = 13: 135 -> 84 VGPRs) but measured
    // no faster at Nq = 12..15 and 10% slower at Nq = 16 (E = 262144).
    constexpr bool FENCE_R = sizeof(TC) == 8 && NQ >= 11;
    constexpr bool FENCE_S = sizeof(TC) == 8 && NQ >= 12;
    // FP64 at Nq = 13: the u column is kept live to the end of the element, as
    // the CG form (DOT) keeps it; the register allocator then fits the kernel
    // in 154 VGPRs (three waves per SIMD) instead of 182 (two)
    constexpr bool PIN_U = !DOT && sizeof(TC) == 8 && NQ == 13;
    constexpr int IOR = GE > 0 ? GE : 1, IOC = QE > 0 ? QE : 1;
    __shared__ TC sIe[TLDS ? HG : 1][HQ];
    __shared__ TC sIo[TLDS ? IOR : 1][IOC];
    TC rIe[TLDS ? 1 : HG][HQ], rIo[TLDS ? 1 : IOR][IOC];
    double tv0 = 0.0, tv1 = 0.0;
    if constexpr (TLDS) {
        interp_pair_load<NQ>(I1d, L, tv0, tv1);
        __builtin_amdgcn_sched_barrier(0);
    } else {
        interp_half_tables<NQ>(I1d, rIe, rIo);
    }
    const TC(*Ie)[HQ] = TLDS ? sIe : rIe;
    const TC(*Io)[IOC] = TLDS ? sIo : rIo;

    // the u column of lane (i,j) and this lane's pieces of the element's wJ
    const int li = L % NQ, lj = L / NQ;
    const bool gll = L < NC;
    // 16-bit fields: the element's u block is fetched in 16-byte pieces by all
    // lanes and turned into columns through LDS (B is free until the
    // s-interpolation), instead of Nq 2-byte loads per lane
    constexpr bool USTAGE = sizeof(TV) == 2 && (NP % 8) == 0;
    constexpr int UPL = (NP / 8 + NT - 1) / NT;   // pieces per lane
    using R16 = typename raw_vec<16>::type;
    TC uc[NQ];
    R16 upc[USTAGE ? UPL : 1];
    if constexpr (USTAGE) {
        const R16 *src = reinterpret_cast<const R16 *>(u + e * NP);
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int t = L + q * NT;
            upc[q] = t < NP / 8 ? src[t] : R16{};
        }
    } else {
        // every lane loads (lanes without a column read column 0 and never
        // use it): a select after each 16-bit load made the compiler branch
        // around it and wait for it, one round trip per value
        const int64_t base = e * NP + (gll ? L : 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k) uc[k] = ld<TC>(u, base + k * NC);
    }
    // wJ pieces: 8-byte pieces for FP64 data, dwords otherwise (16-bit values:
    // the dwords wholly inside the element plus a half-filled first one; a
    // last value sharing its dword with the next element is fetched alone)
    constexpr int PB = sizeof(TG) == 8 ? 8 : 4;                  // piece bytes
    constexpr int VPP = PB / static_cast<int>(sizeof(TG));       // values per piece
    constexpr int NPC = NPG / VPP + 1;
    constexpr int PPL = (NPC + NT - 1) / NT;               // pieces per lane
    using Piece = typename std::conditional<PB == 8, unsigned long long, uint32_t>::type;
    const int64_t v0 = e * NPG;
    const int64_t p0 = v0 / VPP, np = (v0 + NPG) / VPP - p0;
    const int off = static_cast<int>(v0 - p0 * VPP);
    const bool tail = VPP == 2 && ((v0 + NPG) % 2) == 1;
    // The loads are unconditional (clamped indices; the surplus is never
    // stored): with a load under a lane condition the compiler no longer counts
    // the requests in flight and waits for all of them before the t-interpolation.
    Piece wst[PPL];
    uint16_t wlast = 0;
    {
        const Piece *wp = reinterpret_cast<const Piece *>(wJ) + p0;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int t = L + q * NT;
            wst[q] = __builtin_nontemporal_load(wp + (t < np ? t : np - 1));
        }
        if constexpr (VPP == 2) wlast = reinterpret_cast<const uint16_t *>(wJ)[v0 + NPG - 1];
    }

    if constexpr (USTAGE) {
#pragma unroll
        for (int q = 0; q < UPL; ++q) {
            const int t = L + q * NT;
            if (t < NP / 8) {
                TV tmp[8];
                __builtin_memcpy(tmp, &upc[q], 16);
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int n = t * 8 + v;
                    const int k = n / NC, r = n - k * NC;
                    sB[k * NQ * P + (r / NQ) * P + r % NQ] = to_compute(tmp[v], TC{});
                }
            }
        }
        __syncthreads();
        if (gll) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = sB[k * NQ * P + lj * P + li];
        }
    }

    if constexpr (TLDS) {
        interp_pair_store<NQ>(sIe, sIo, L, tv0, tv1);
        __syncthreads();
    }

    // t-interpolation: lanes (i,j)
    if (gll) {
        TC z[NG];
        line_interp<NQ>(uc, z, Ie, Io);
#pragma unroll
        for (int c = 0; c < NG; ++c) sA[c * SA + lj * P + li] = z[c];
    }
    __syncthreads();

    // s-interpolation: lines (i,c)
#pragma unroll
    for (int pass = 0; pass < (NQ * NG + NT - 1) / NT; ++pass) {
        const int line = L + pass * NT;
        if (line < NQ * NG) {
            const int i = line % NQ, c = line / NQ;
            TC x[NQ], z[NG];
#pragma unroll
            for (int m = 0; m < NQ; ++m) x[m] = sA[c * SA + m * P + i];
            if constexpr (FENCE_S) asm volatile("" ::: "memory");
            line_interp<NQ>(x, z, Ie, Io);
#pragma unroll
            for (int b = 0; b < NG; ++b) sB[c * SB + b * P + i] = z[b];
        }
    }
    __syncthreads();   // A is free: stage wJ there
    if constexpr (!REMAP) {
        Piece *sw = reinterpret_cast<Piece *>(sA);
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int t = L + q * NT;
            if (t < np) sw[t] = wst[q];
        }
        if (tail && L == 0) reinterpret_cast<uint16_t *>(sA)[off + NPG - 1] = wlast;
    } else {
        TG *sw = reinterpret_cast<TG *>(sA);
        // value v of the element (its stored layout) -> row (c, b), entry a
        auto put = [&](int v, TG val) {
            const int q = v / W, c = (q / (NG * NG)) * W + v % W, col = q % (NG * NG);
            sw[(c * NG + col / NG) * PW + col % NG] = val;
        };
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int t = L + q * NT;
            if (t < np) {
                TG vals[VPP];
                __builtin_memcpy(vals, &wst[q], sizeof(Piece));
#pragma unroll
                for (int r = 0; r < VPP; ++r) {
                    const int v = t * VPP + r - off;
                    if (v >= 0 && v < NPG) put(v, vals[r]);
                }
            }
        }
        if constexpr (VPP == 2) {
            if (tail && L == 0) {
                TG last;
                __builtin_memcpy(&last, &wlast, sizeof(TG));
                put(NPG - 1, last);
            }
        }
    }
    __syncthreads();

    // r-direction: lines (b,c): interpolate, scale by wJ, project, in place
    {
        const TG *sw = reinterpret_cast<const TG *>(sA) + (REMAP ? 0 : off);
#pragma unroll
        for (int pass = 0; pass < (NG * NG + NT - 1) / NT; ++pass) {
            const int line = L + pass * NT;
            if (line < NG * NG) {
                const int b = line % NG, c = line / NG;
                TC x[NQ], z[NG], w[NQ];
                TC *row = sB + c * SB + b * P;
#pragma unroll
                for (int m = 0; m < NQ; ++m) x[m] = row[m];
                if constexpr (FENCE_R) asm volatile("" ::: "memory");
                line_interp<NQ>(x, z, Ie, Io);
#pragma unroll
                for (int a = 0; a < NG; ++a)
                    z[a] *= to_compute(sw[REMAP ? (c * NG + b) * PW + a : geo_offset(a + NG * b, c, NG, W)], TC{});
                if constexpr (FENCE_R) asm volatile("" ::: "memory");
                line_project<NQ>(z, w, Ie, Io);
#pragma unroll
                for (int m = 0; m < NQ; ++m) row[m] = w[m];
            }
        }
    }
    __syncthreads();

    // with beta != 0 the old y column of lane (i,j) is requested here, so its
    // latency hides behind the s-projection
    TC yold[NQ];
    if (beta != TC(0) && gll) {
        const int64_t base = e * NP + L;
#pragma unroll
        for (int k = 0; k < NQ; ++k) yold[k] = static_cast<TC>(y[base + k * NC]);
    }

    // s-projection: lines (i,c) -> A[c][j][i]
#pragma unroll
    for (int pass = 0; pass < (NQ * NG + NT - 1) / NT; ++pass) {
        const int line = L + pass * NT;
        if (line < NQ * NG) {
            const int i = line % NQ, c = line / NQ;
            TC v[NG], w[NQ];
#pragma unroll
            for (int b = 0; b < NG; ++b) v[b] = sB[c * SB + b * P + i];
            if constexpr (FENCE_S) asm volatile("" ::: "memory");
            line_project<NQ>(v, w, Ie, Io);
#pragma unroll
            for (int j = 0; j < NQ; ++j) sA[c * SA + j * P + i] = w[j];
        }
    }
    __syncthreads();

    // t-projection: lanes (i,j) -> y[k][j][i]
    double dp = 0.0;
    if (gll) {
        TC v[NG], w[NQ];
#pragma unroll
        for (int c = 0; c < NG; ++c) v[c] = sA[c * SA + lj * P + li];
        line_project<NQ>(v, w, Ie, Io);
        const int64_t base = e * NP + L;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            TC r = w[k] * oscale;
            const int64_t idx = base + k * NC;
            if (beta != TC(0)) r += beta * yold[k];
            y[idx] = static_cast<TY>(r);
            if constexpr (DOT) dp += static_cast<double>(uc[k]) * static_cast<double>(r);
        }
        if constexpr (PIN_U) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) asm volatile("" ::"v"(uc[k]));
        }
    }
    if constexpr (DOT) {
        static_assert(std::is_same<TV, double>::value || std::is_same<TV, float>::value,
                      "element partials of FP64 or FP32 fields");
#pragma unroll
        for (int o = kWave / 2; o > 0; o >>= 1) dp += __shfl_xor(dp, o);
        if constexpr (NT == kWave) {
            if (L == 0) part[e] = dp;
        } else {
            // one partial per wave, summed in wave order
            __shared__ double s_red[NT / kWave];
            if (L % kWave == 0) s_red[L / kWave] = dp;
            __syncthreads();
            if (L == 0) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < NT / kWave; ++w) t += s_red[w];
                part[e] = t;
            }
        }
    }
}

template <int NQ, class TG, class TV>
hipError_t bp10t_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    if (a.E < 1) return hipSuccess;
    if (a.part && !(std::is_same<TV, double>::value || (std::is_same<TV, float>::value && NQ <= 8)))
        return hipErrorInvalidValue;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    // one workgroup per element; a grid cap splits the elements over launches
    int64_t chunk = a.grid_cap > 0 ? a.grid_cap : a.E;
    if (chunk > max_grid(bp10t_threads(NQ))) chunk = max_grid(bp10t_threads(NQ));
    for (int64_t e0 = 0; e0 < a.E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(a.E - e0 < chunk ? a.E - e0 : chunk);
        if constexpr (std::is_same<TV, double>::value || (std::is_same<TV, float>::value && NQ <= 8)) {
            if (a.part) {
                hipLaunchKernelGGL((bp10t_kernel<NQ, TG, TV, true>), dim3(grid), dim3(bp10t_threads(NQ)), 0, s, a.E, a.I1d,
                                   static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u),
                                   static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale, a.part, e0);
                continue;
            }
        }
        hipLaunchKernelGGL((bp10t_kernel<NQ, TG, TV>), dim3(grid), dim3(bp10t_threads(NQ)), 0, s, a.E, a.I1d,
                           static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u),
                           static_cast<TY *>(a.y), static_cast<TC>(a.beta), oscale, nullptr, e0);
    }
    return hipGetLastError();
}

}  // namespace fem
