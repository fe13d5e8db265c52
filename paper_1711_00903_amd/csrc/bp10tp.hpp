// bp10tp.hpp -- BP1.0 mass operator in persistent form: the line-per-lane
// kernel of bp10t.hpp (one element per workgroup at a time, every
// one-direction contraction of Alg. 1-3 done by a lane that owns a whole line,
// the element turned between directions through LDS), looping over elements
// e, e + G, e + 2G, ... (G the grid).  Before a workgroup works on an element
// it requests the next element's u and wJ, so each wave keeps HBM requests in
// flight through its LDS and ALU phases; in the one-shot kernel a wave's
// requests for an element are issued only when the previous workgroup on its
// slot has finished.  The cost is the registers of one more element's loads
// (Nq 4-byte or 8-byte values of u, or 16-byte pieces for 16-bit fields, and
// ceil((Ng^3 / values per piece + 1) / lanes) wJ pieces), so the form is used
// only where it measured faster.
#pragma once

#include "bp10t.hpp"

namespace fem {

template <int NQ, class TG, class TV, bool DOT = false>
__global__ __launch_bounds__(bp10t_threads(NQ)) void bp10tp_kernel(
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
    // LDS volumes, wJ staging, line products and fences as in bp10t_kernel;
    // the half tables are in registers (Nq <= 11)
    static_assert(NQ <= 11, "persistent form for Nq <= 11");
    constexpr int P = bp10t_row(NQ, sizeof(TC));
    constexpr int SA = NQ * P;                   // slab of A: [j][i]
    constexpr int SB = NG * P;                   // slab of B: [b][i]
    constexpr int W = geo_vec(NG, sizeof(TG));   // interleave of the geometric layout
    constexpr int NT = bp10t_threads(NQ);
    static_assert(NC <= NT, "one lane per GLL column");
    static_assert(!bp10t_remap_w(NG, static_cast<int>(sizeof(TG))), "wJ staged as stored");
    constexpr int WBYTES = NPG * static_cast<int>(sizeof(TG)) + 8;   // (+ misalignment slack)
    constexpr int AV = NG * SA;
    constexpr int A_VALUES = AV * static_cast<int>(sizeof(TC)) > WBYTES ? AV
                                                                        : (WBYTES + sizeof(TC) - 1) / sizeof(TC);
    __shared__ __align__(16) TC sA[A_VALUES];
    __shared__ __align__(16) TC sB[NG * SB];

    const int L = threadIdx.x;
    constexpr bool FENCE_R = sizeof(TC) == 8 && NQ >= 11;
    constexpr int IOC = QE > 0 ? QE : 1;
    TC Ie[HG][HQ], Io[GE > 0 ? GE : 1][IOC];
    interp_half_tables<NQ>(I1d, Ie, Io);

    const int li = L % NQ, lj = L / NQ;
    const bool gll = L < NC;
    // 16-bit fields: the element's u block is fetched in 16-byte pieces by all
    // lanes and turned into columns through LDS (B is free until the
    // s-interpolation), instead of Nq 2-byte loads per lane
    constexpr bool USTAGE = sizeof(TV) == 2 && (NP % 8) == 0;
    constexpr int UPL = (NP / 8 + NT - 1) / NT;   // pieces per lane
    using R16 = typename raw_vec<16>::type;
    // wJ pieces: 8-byte pieces for FP64 data, dwords otherwise (16-bit values:
    // the dwords wholly inside the element plus a half-filled first one; a
    // last value sharing its dword with the next element is fetched alone)
    constexpr int PB = sizeof(TG) == 8 ? 8 : 4;                  // piece bytes
    constexpr int VPP = PB / static_cast<int>(sizeof(TG));       // values per piece
    constexpr int NPC = NPG / VPP + 1;
    constexpr int PPL = (NPC + NT - 1) / NT;               // pieces per lane
    using Piece = typename std::conditional<PB == 8, unsigned long long, uint32_t>::type;

    // what one element reads from HBM: the u column of lane (i,j) (or its
    // 16-byte pieces of u) and this lane's pieces of the element's wJ
    struct In {
        TC uc[USTAGE ? 1 : NQ];
        R16 upc[USTAGE ? UPL : 1];
        Piece wst[PPL];
        uint16_t wlast;
    };
    auto fetch = [&](int64_t el, In &in) {
        if constexpr (USTAGE) {
            const R16 *src = reinterpret_cast<const R16 *>(u + el * NP);
#pragma unroll
            for (int q = 0; q < UPL; ++q) {
                const int t = L + q * NT;
                in.upc[q] = t < NP / 8 ? src[t] : R16{};
            }
        } else {
            // every lane loads (lanes without a column read column 0 and never
            // use it): a select after each 16-bit load made the compiler branch
            // around it and wait for it, one round trip per value
            const int64_t base = el * NP + (gll ? L : 0);
#pragma unroll
            for (int k = 0; k < NQ; ++k) in.uc[k] = ld<TC>(u, base + k * NC);
        }
        // The loads are unconditional (clamped indices; the surplus is never
        // stored): with a load under a lane condition the compiler no longer
        // counts the requests in flight and waits for all of them before the
        // t-interpolation.
        const int64_t v0 = el * NPG;
        const int64_t p0 = v0 / VPP, np = (v0 + NPG) / VPP - p0;
        const Piece *wp = reinterpret_cast<const Piece *>(wJ) + p0;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int t = L + q * NT;
            in.wst[q] = __builtin_nontemporal_load(wp + (t < np ? t : np - 1));
        }
        in.wlast = 0;
        if constexpr (VPP == 2) in.wlast = reinterpret_cast<const uint16_t *>(wJ)[v0 + NPG - 1];
    };

    __shared__ double s_red[NT / kWave];
    auto element = [&](int64_t e, In &in) {
        const int64_t v0 = e * NPG;
        const int64_t p0 = v0 / VPP, np = (v0 + NPG) / VPP - p0;
        const int off = static_cast<int>(v0 - p0 * VPP);
        const bool tail = VPP == 2 && ((v0 + NPG) % 2) == 1;
        TC uc[NQ];
        if constexpr (USTAGE) {
#pragma unroll
            for (int q = 0; q < UPL; ++q) {
                const int t = L + q * NT;
                if (t < NP / 8) {
                    TV tmp[8];
                    __builtin_memcpy(tmp, &in.upc[q], 16);
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
        } else {
#pragma unroll
            for (int k = 0; k < NQ; ++k) uc[k] = in.uc[k];
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
                line_interp<NQ>(x, z, Ie, Io);
#pragma unroll
                for (int b = 0; b < NG; ++b) sB[c * SB + b * P + i] = z[b];
            }
        }
        __syncthreads();   // A is free: stage wJ there
        {
            Piece *sw = reinterpret_cast<Piece *>(sA);
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
                const int t = L + q * NT;
                if (t < np) sw[t] = in.wst[q];
            }
            if (tail && L == 0) reinterpret_cast<uint16_t *>(sA)[off + NPG - 1] = in.wlast;
        }
        __syncthreads();

        // r-direction: lines (b,c): interpolate, scale by wJ, project, in place
        {
            const TG *sw = reinterpret_cast<const TG *>(sA) + off;
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
                        z[a] *= to_compute(sw[geo_offset(a + NG * b, c, NG, W)], TC{});
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
    };

    // elements e0 + blockIdx.x + k * gridDim.x below E; the grid is at most
    // E - e0 workgroups, so every workgroup has a first element.  The last
    // element's prefetch re-reads that element (in bounds, not used).
    int64_t e = e0 + blockIdx.x;
    In cur, nxt;
    fetch(e, cur);
    for (;;) {
        const int64_t en = e + gridDim.x;
        const bool more = en < E;
        fetch(more ? en : e, nxt);
        element(e, cur);
        if (!more) break;
        e = en;
        cur = nxt;
        __syncthreads();   // the t-projection's reads of A before the next t-interpolation's writes
    }
}

// Where the persistent form replaces the one-shot kernel (MI355X, E = 262144,
// library sweeps of both, same bits): FP32 or 16-bit fields at Nq = 9..11
// (FP32 1.06-1.13x, BF16 1.13-1.30x, BF16 wJ with FP32 fields 1.08-1.21x)
// and FP64 fields with FP32 or 16-bit wJ at Nq = 10..11 (1.10-1.11x).
// Elsewhere the one-shot kernel keeps enough elements in flight per CU: FP64
// fields and factors 0.88-1.03x at Nq = 7..11, every precision 0.93-1.07x at
// Nq = 8, narrow wJ with FP64 fields 1.01x at Nq = 9.
constexpr bool bp10tp_use(int nq, int gbytes, int vbytes)
{
    return (vbytes < 8 && nq >= 9 && nq <= 11) || (vbytes == 8 && gbytes < 8 && nq >= 10 && nq <= 11);
}

// default grid: this many times the workgroups resident at once (each then
// takes about E / grid elements; 4x and 8x measured best, 1x 5-25% slower)
constexpr int kBp10tpGridMult = 8;

// workgroups of KERNEL resident on the current device at once, taken once per
// kernel
template <auto KERNEL>
int64_t bp10tp_resident(int threads)
{
    static const int64_t n = [threads]() -> int64_t {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, KERNEL, threads, 0) != hipSuccess || cus < 1 || per < 1)
            return 0;
        return static_cast<int64_t>(cus) * per;
    }();
    return n;
}

// one launch of grid_cap workgroups (0: kBp10tpGridMult times those resident
// at once), capped at E
template <int NQ, class TG, class TV>
hipError_t bp10tp_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr bool PART = std::is_same<TV, double>::value || (std::is_same<TV, float>::value && NQ <= 8);
    if (a.E < 1) return hipSuccess;
    if (a.part && !PART) return hipErrorInvalidValue;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    const int thr = bp10t_threads(NQ);
    auto launch = [&](auto kernel, int64_t resident, double *part) -> hipError_t {
        int64_t grid = a.grid_cap > 0 ? a.grid_cap : kBp10tpGridMult * resident;
        if (grid < 1) return hipErrorInvalidConfiguration;   // occupancy query failed
        if (grid > a.E) grid = a.E;
        if (grid > max_grid(thr)) grid = max_grid(thr);
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(grid)), dim3(thr), 0, s, a.E, a.I1d,
                           static_cast<const TG *>(a.wJ), static_cast<const TV *>(a.u), static_cast<TY *>(a.y),
                           static_cast<TC>(a.beta), oscale, part, int64_t{0});
        return hipGetLastError();
    };
    if constexpr (PART) {
        if (a.part)
            return launch(bp10tp_kernel<NQ, TG, TV, true>, bp10tp_resident<bp10tp_kernel<NQ, TG, TV, true>>(thr),
                          a.part);
    }
    return launch(bp10tp_kernel<NQ, TG, TV>, bp10tp_resident<bp10tp_kernel<NQ, TG, TV>>(thr), nullptr);
}

}  // namespace fem
