// bp35t.hpp -- BP3.5 collocated stiffness at high degree, one element per
// workgroup of ceil(Nq^2 / 64) waves, every one-direction product done by the
// lane that owns a whole line (Alg. 4).
//
// The GLL derivative matrix is centro-antisymmetric, D[a][m] = -D[Nq-1-a][Nq-1-m],
// so each line product and its transpose run in even-odd form on half tables
// (lines.hpp), held in LDS: at these degrees the registers go to the lines and
// the prefetched geometric factors.  Lane p + Nq k owns r-line (p,k) and
// s-line (p,k) of slab k; lane i + Nq j owns GLL column (i,j).  Two LDS volumes
// (Nq^3 each, rows padded):
//   columns        u column (registers)                -> V0 = U[k][j][i]
//   r-derivative   lines (j,k) of V0                   -> V1 = QR
//   s-derivative   lines (i,k) of V0, in place         -> V0 = QS
//   metric         columns (i,j): qt = D u (registers); (wr,ws,wt) = G (qr,qs,qt);
//                  WR over QR, WS over QS; vt = D^T wt (+ lambda wJ u) in registers
//   transposes     s-lines of V0 and r-lines of V1, in place (D^T)
//   columns        y = V0 + V1 + vt
// Compared with the column kernel (bp35.hpp, a lane per column reading whole
// LDS lines for every output) this moves one LDS write and one read per point
// and direction, and needs two volumes instead of three.
#pragma once

#include "fem_device.hpp"
#include "launch.hpp"
#include "lines.hpp"
#include "tiles.hpp"

namespace fem {

constexpr int bp35t_threads(int nq) { return round_up_wave(nq * nq); }

// Waves per SIMD asked of the register allocator: two up to Nq = 13, where
// that costs no spills (the allocator would otherwise take a few extra
// registers and run one wave per SIMD).
constexpr int bp35t_min_waves(int nq) { return nq <= 13 ? 2 : 1; }

template <int NQ, class TG, class TV>
__global__ __launch_bounds__(bp35t_threads(NQ))
__attribute__((amdgpu_waves_per_eu(bp35t_min_waves(NQ)))) void bp35t_kernel(
    int64_t E, const double *__restrict__ D1d, const TG *__restrict__ G, const TG *__restrict__ wJ,
    typename compute_pair<TG, TV>::type lambda, const TV *__restrict__ u,
    typename output_of<TV>::type *__restrict__ y, typename compute_pair<TG, TV>::type beta,
    typename compute_pair<TG, TV>::type oscale, int64_t e0)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int HQ = (NQ + 1) / 2, QE = NQ / 2;
    constexpr int P = lds_row(NQ, sizeof(TC));   // row length of both volumes
    constexpr int S = NQ * P;                    // slab
    constexpr int VOL = NQ * S;
    constexpr int W = geo_vec(NQ, sizeof(TG));   // slabs per vector load of geometric data
    constexpr int NV = NQ / W;
    // groups of W slabs of factors requested ahead of use (two in FP64 arithmetic
    // beyond Nq = 11, where three no longer fit in registers)
    constexpr int GPRE = NV < 3 ? NV : (sizeof(TC) == 8 && NQ >= 12 ? 2 : 3);
    static_assert(NQ >= 2 && NC <= bp35t_threads(NQ), "one lane per GLL column");
    // From Nq = 12: an empty asm with a memory clobber between two line
    // products makes the second read its LDS half tables again; otherwise the
    // compiler holds the first product's table values in registers for the
    // second, which cost a wave per SIMD (FP64, measured at E = 65536: Nq = 12
    // 4.0 -> 5.1, Nq = 14 2.6 -> 5.1, Nq = 16 3.3 -> 5.7 TB/s; FP32 arithmetic
    // with 16-bit storage at E = 262144: Nq = 13 3.3 -> 2.4 ms, Nq = 14 3.8 ->
    // 3.0, Nq = 15 4.5 -> 3.7, with FP32 storage unchanged).
    constexpr bool FENCE = NQ >= 12;

    __shared__ __align__(16) TC V0[VOL];
    __shared__ __align__(16) TC V1[VOL];
    __shared__ TC sDp[QE][HQ];
    __shared__ TC sDm[HQ][QE];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;
    const bool own = L < NC;                     // owns column (ci,cj) and lines (lp, lk)
    // lanes beyond the columns re-read the first column of their own wave (every
    // wave holds at least one) and never store: no request of a wave touches a
    // line outside its own columns
    const int gcol = own ? L : (L & ~(kWave - 1));
    const int ci = gcol % NQ, cj = gcol / NQ;
    const int lp = ci, lk = cj;

    // Requests, oldest first: this lane's pair of table entries, the u column,
    // the first GPRE groups of the column's factors.  Every lane issues them
    // (a load under a lane condition makes the compiler wait for it in place).
    double td0, td1;
    deriv_pair_load<NQ>(D1d, L, td0, td1);
    __builtin_amdgcn_sched_barrier(0);
    TV uraw[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) uraw[k] = u[e * NP + gcol + k * NC];
    __builtin_amdgcn_sched_barrier(0);
    const TG *Ge = G + e * (6 * NP) + gcol * W;
    packed_vec<W, TG> gq[NV][6];
#pragma unroll
    for (int q = 0; q < GPRE; ++q)
#pragma unroll
        for (int f = 0; f < 6; ++f) gq[q][f].stream(Ge + f * NP + q * NC * W);
    __builtin_amdgcn_sched_barrier(0);

    deriv_pair_store<NQ>(sDp, sDm, L, td0, td1);
    TC uc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) uc[k] = to_compute(uraw[k], TC{});
    if (own) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) V0[k * S + cj * P + ci] = uc[k];
    }
    __syncthreads();
    const TC(*Dp)[HQ] = sDp;
    const TC(*Dm)[QE] = sDm;

    // r-derivative: row (j = lp) of slab lk -> V1
    if (own) {
        TC x[NQ], z[NQ];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[lk * S + lp * P + m];
        line_deriv<NQ>(x, z, Dp, Dm);
#pragma unroll
        for (int a = 0; a < NQ; ++a) V1[lk * S + lp * P + a] = z[a];
    }
    __syncthreads();
    // s-derivative: column (i = lp) of slab lk, in place in V0
    if (own) {
        TC x[NQ], z[NQ];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[lk * S + m * P + lp];
        line_deriv<NQ>(x, z, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NQ; ++b) V0[lk * S + b * P + lp] = z[b];
    }
    __syncthreads();

    // metric step on column (ci,cj); the t-direction stays in registers
    TC vt[NQ];
    if (own) {
        const int o = cj * P + ci;
        TC qt[NQ], wt[NQ];
        line_deriv<NQ>(uc, qt, Dp, Dm);
        if constexpr (FENCE) asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            if (k % W == 0 && k / W + GPRE < NV) {
#pragma unroll
                for (int f = 0; f < 6; ++f) gq[k / W + GPRE][f].stream(Ge + f * NP + (k / W + GPRE) * NC * W);
            }
            const TC qr = V1[k * S + o], qs = V0[k * S + o];
            const TC grr = gq[k / W][0].template get<TC>(k % W);
            const TC grs = gq[k / W][1].template get<TC>(k % W);
            const TC grt = gq[k / W][2].template get<TC>(k % W);
            const TC gss = gq[k / W][3].template get<TC>(k % W);
            const TC gst = gq[k / W][4].template get<TC>(k % W);
            const TC gtt = gq[k / W][5].template get<TC>(k % W);
            V1[k * S + o] = grr * qr + grs * qs + grt * qt[k];
            V0[k * S + o] = grs * qr + gss * qs + gst * qt[k];
            wt[k] = grt * qr + gst * qs + gtt * qt[k];
        }
        if constexpr (FENCE) asm volatile("" ::: "memory");
        line_deriv_t<NQ>(wt, vt, Dp, Dm);
        if (lambda != TC(0)) {
            // u is fetched again (from cache) rather than kept live through the
            // metric step
#pragma unroll
            for (int k = 0; k < NQ; ++k)
                vt[k] += lambda * ld<TC>(wJ, e * NP + geo_offset(gcol, k, NQ, W)) * ld<TC>(u, e * NP + gcol + k * NC);
        }
    }
    // the old y column when beta != 0, requested before the transposes
    TC yold[NQ];
    if (beta != TC(0) && own) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) yold[k] = static_cast<TC>(y[e * NP + L + k * NC]);
    }
    __syncthreads();

    // transposes, in place: s-line (lp,lk) of WS and r-line (lp,lk) of WR
    if (own) {
        TC v[NQ], w[NQ];
#pragma unroll
        for (int b = 0; b < NQ; ++b) v[b] = V0[lk * S + b * P + lp];
        line_deriv_t<NQ>(v, w, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NQ; ++b) V0[lk * S + b * P + lp] = w[b];
        if constexpr (FENCE) asm volatile("" ::: "memory");
#pragma unroll
        for (int a = 0; a < NQ; ++a) v[a] = V1[lk * S + lp * P + a];
        line_deriv_t<NQ>(v, w, Dp, Dm);
#pragma unroll
        for (int a = 0; a < NQ; ++a) V1[lk * S + lp * P + a] = w[a];
    }
    __syncthreads();

    // y column (ci,cj) = r and s terms from LDS + t term from registers
    if (own) {
        const int o = cj * P + ci;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            TC r = (V0[k * S + o] + V1[k * S + o] + vt[k]) * oscale;
            if (beta != TC(0)) r += beta * yold[k];
            y[e * NP + L + k * NC] = static_cast<TY>(r);
        }
    }
}

template <int NQ, class TG, class TV>
hipError_t bp35t_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    if (a.E < 1) return hipSuccess;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    // one workgroup per element; a grid cap splits the elements over launches
    int64_t chunk = a.grid_cap > 0 ? a.grid_cap : a.E;
    if (chunk > max_grid(bp35t_threads(NQ))) chunk = max_grid(bp35t_threads(NQ));
    for (int64_t e0 = 0; e0 < a.E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(a.E - e0 < chunk ? a.E - e0 : chunk);
        hipLaunchKernelGGL((bp35t_kernel<NQ, TG, TV>), dim3(grid), dim3(bp35t_threads(NQ)), 0, s, a.E, a.D1d,
                           static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                           static_cast<TC>(a.lambda), static_cast<const TV *>(a.u), static_cast<TY *>(a.y),
                           static_cast<TC>(a.beta), oscale, e0);
    }
    return hipGetLastError();
}

}  // namespace fem
