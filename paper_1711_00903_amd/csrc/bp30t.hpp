// bp30t.hpp -- BP3.0 de-aliased stiffness, one element per workgroup of
// ceil(Ng^2 / 64) waves, one-direction contractions done by the
// lane that owns a whole line (Alg. 5 with the interpolation and projection
// of Alg. 1-2).
//
// Lane (a,b) of the Gauss grid owns column (a,b) for the metric step and
// (up to Ng = 9) requests all 6 Ng geometric factors of that column before the
// first barrier, so the element's whole geometric read (81% of its bytes) is
// in flight while the field is interpolated.  Every other step is a line product
// with a uniform half table (lines.hpp), and the element turns between line
// directions through LDS:
//   t-interpolation  lanes (i,j): u column (registers)      -> A[c][j][i]
//   s-interpolation  lines (i,c): A[c][*][i]                -> B[c][b][i]
//   r-interpolation  lines (b,c): B[c][b][*]                -> U[c][b][a]   (u~ at Gauss points)
//   r-, s-derivative lines (b,c) and (a,c) of U             -> QR, QS
//   metric           columns (a,b): t-derivative of the U column, then
//                    (wr,ws,wt) = G (qr,qs,qt); WR, WS over QR, QS; the column's
//                    D~^T wt (+ lambda wJ u~) over its U column          -> V
//   s-transpose      lines (a,c): WS[c][*][a] <- D~^T WS[c][*][a]
//   r-transpose      lines (b,c): D~^T WR[c][b][*] + V + WS, then projected -> X[c][b][i]
//   s-projection     lines (i,c): X[c][*][i]                -> Y[c][j][i]
//   t-projection     lanes (i,j): Y[*][j][i]                -> y[k][j][i]
// Three LDS volumes (Ng^3 each, rows padded) are reused:
//   V0: A, then QR / WR, then Y;  V1: B, then QS / WS;  V2: U, then V, then X.
// The interpolation and derivative half tables are live in different phases
// (only both in the r-transpose), which keeps the registers for the factors.
#pragma once

#include "bp35.hpp"
#include "lines.hpp"

namespace fem {

constexpr int bp30t_threads(int nq) { return round_up_wave((nq + 1) * (nq + 1)); }

template <int NQ, class TG, class TV>
__global__ __launch_bounds__(bp30t_threads(NQ)) void bp30t_kernel(
    int64_t E, const double *__restrict__ I1d, const double *__restrict__ Dgl, const TG *__restrict__ G,
    const TG *__restrict__ wJ, typename compute_pair<TG, TV>::type lambda, const TV *__restrict__ u,
    typename output_of<TV>::type *__restrict__ y, typename compute_pair<TG, TV>::type beta,
    typename compute_pair<TG, TV>::type oscale, int64_t e0)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    constexpr int NG = NQ + 1;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int NCG = NG * NG;
    constexpr int NPG = NCG * NG;
    constexpr int HG = (NG + 1) / 2, HQ = (NQ + 1) / 2, GE = NG / 2, QE = NQ / 2;
    constexpr int P = lds_row(NG, sizeof(TC));   // row length of every volume
    constexpr int S = NG * P;                    // slab
    constexpr int VOL = NG * S;
    constexpr int W = geo_vec(NG, sizeof(TG));
    static_assert(NCG <= bp30t_threads(NQ), "one lane per Gauss column");

    __shared__ __align__(16) TC V0[VOL];
    __shared__ __align__(16) TC V1[VOL];
    __shared__ __align__(16) TC V2[VOL];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;
    const bool col = L < NCG;                    // owns Gauss column (ca, cb)
    const int ca = L % NG, cb = L / NG;

    // the u column of lane (i,j) and the 6 Ng factors of Gauss column (ca,cb).
    // Every lane loads (lanes beyond the columns re-read another column and never
    // use it): under a lane condition the compiler widens a narrow value inside the
    // branch and waits for it there, one load at a time.  The u column is
    // requested first and waited for only after the factor requests are out.
    const bool gll = L < NC;
    const int li = L % NQ, lj = L / NQ;
    // Half tables: in registers for small Nq, in LDS beyond (the lines then
    // need the registers); the LDS copies are fetched ahead of the element's
    // loads and stored once those are issued.  Measured crossovers: FP32
    // arithmetic from Nq = 11; FP64 arithmetic from Nq = 10, together with one
    // slab of factors ahead and the table reads of consecutive line products
    // kept apart (FENCE, below), which fit the kernel in two waves per SIMD
    // (Nq = 10: 3.9 -> 4.5 TB/s, Nq = 12: 3.0 -> 4.1 TB/s at E = 65536).
    constexpr bool FENCE = sizeof(TC) == 8 && NQ >= 10;
    // FP32 arithmetic at Nq = 14: the same fences without the FP64 prefetch and
    // table choices (230 -> 150 VGPRs, two -> three waves per SIMD; 12% faster
    // at E = 262144 with FP32, BF16 and FP16 storage; at Nq = 12, 13, 15 and 16
    // they cut registers too but measured 4-10% slower)
    constexpr bool FENCE32 = sizeof(TC) == 4 && NQ == 14;
    constexpr bool TLDS = FENCE || NQ > 12 || NQ == 11 || (NQ == 12 && sizeof(TC) == 4);
    constexpr int QEC = QE > 0 ? QE : 1;
    __shared__ TC sIe[TLDS ? HG : 1][HQ];
    __shared__ TC sIo[TLDS ? GE : 1][QEC];
    __shared__ TC sDp[TLDS ? GE : 1][HG];
    __shared__ TC sDm[TLDS ? HG : 1][GE];
    double ti0 = 0.0, ti1 = 0.0, td0 = 0.0, td1 = 0.0;
    if constexpr (TLDS) {
        interp_pair_load<NQ>(I1d, L, ti0, ti1);
        deriv_pair_load<NG>(Dgl, L, td0, td1);
        __builtin_amdgcn_sched_barrier(0);
    }
    TV uraw[NQ];
    {
        const int64_t base = e * NP + (gll ? L : 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k) uraw[k] = u[base + k * NC];
    }
    __builtin_amdgcn_sched_barrier(0);
    // up to Ng = 9 every slab of the column's factors is requested here; beyond,
    // the first GPRE slabs, and each later slab GPRE slabs ahead of its use in
    // the metric step (all of them no longer fit in registers).  The factors
    // stay in their stored type until the metric step: a widening right after
    // the load would wait for every request before the first barrier.
    constexpr int GPRE = FENCE ? 1 : (NG <= 9 ? NG : (NG <= 11 ? 4 : (NG <= 16 ? 3 : 2)));
    TG g[6][NG];
    const int64_t gb = e * (6 * NPG);
    // a lane without a column re-reads the first column of its own wave (every
    // wave holds at least one column), so the wave's requests touch no line
    // outside its own columns: with non-temporal loads a re-read of column 0
    // from another wave went to HBM again (+17% of the bytes with BF16 factors)
    const int gcol = col ? L : (L & ~(kWave - 1));
    auto gload = [&](int c) {
#pragma unroll
        for (int f = 0; f < 6; ++f) g[f][c] = nt_load(G + gb + f * NPG + geo_offset(gcol, c, NG, W));
    };
#pragma unroll
    for (int c = 0; c < GPRE; ++c) gload(c);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (TLDS) {
        interp_pair_store<NQ>(sIe, sIo, L, ti0, ti1);
        deriv_pair_store<NG>(sDp, sDm, L, td0, td1);
        __syncthreads();
    }
    TC uc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        uc[k] = to_compute(uraw[k], TC{});
        asm volatile("" : "+v"(uc[k]));   // keeps the u loads out of the branch below
    }

    {
        TC rIe[TLDS ? 1 : HG][HQ], rIo[TLDS ? 1 : GE][QEC];
        if constexpr (!TLDS) interp_half_tables<NQ>(I1d, rIe, rIo);
        const TC(*Ie)[HQ] = TLDS ? sIe : rIe;
        const TC(*Io)[QEC] = TLDS ? sIo : rIo;
        // t-interpolation: lanes (i,j) -> V0 = A[c][j][i]
        if (gll) {
            TC z[NG];
            line_interp<NQ>(uc, z, Ie, Io);
#pragma unroll
            for (int c = 0; c < NG; ++c) V0[c * S + lj * P + li] = z[c];
        }
        __syncthreads();
        // s-interpolation: lines (i,c) -> V1 = B[c][b][i]
        if (L < NQ * NG) {
            const int i = L % NQ, c = L / NQ;
            TC x[NQ], z[NG];
#pragma unroll
            for (int m = 0; m < NQ; ++m) x[m] = V0[c * S + m * P + i];
            line_interp<NQ>(x, z, Ie, Io);
#pragma unroll
            for (int b = 0; b < NG; ++b) V1[c * S + b * P + i] = z[b];
        }
        __syncthreads();
        // r-interpolation: lines (b,c) -> V2 = U[c][b][a]
        if (L < NCG) {
            const int b = L % NG, c = L / NG;
            TC x[NQ], z[NG];
#pragma unroll
            for (int m = 0; m < NQ; ++m) x[m] = V1[c * S + b * P + m];
            line_interp<NQ>(x, z, Ie, Io);
#pragma unroll
            for (int a = 0; a < NG; ++a) V2[c * S + b * P + a] = z[a];
        }
        __syncthreads();
    }

    TC rDp[TLDS ? 1 : GE][HG], rDm[TLDS ? 1 : HG][GE];
    if constexpr (!TLDS) deriv_half_tables<NG>(Dgl, rDp, rDm);
    const TC(*Dp)[HG] = TLDS ? sDp : rDp;
    const TC(*Dm)[GE] = TLDS ? sDm : rDm;
    // r- and s-derivatives of U: lines (b,c) -> V0 = QR, lines (a,c) -> V1 = QS
    if (L < NCG) {
        const int p = L % NG, c = L / NG;
        TC x[NG], z[NG];
#pragma unroll
        for (int m = 0; m < NG; ++m) x[m] = V2[c * S + p * P + m];   // row (b = p)
        line_deriv<NG>(x, z, Dp, Dm);
#pragma unroll
        for (int a = 0; a < NG; ++a) V0[c * S + p * P + a] = z[a];
        // An empty asm with a memory clobber between two line products makes
        // the second read its LDS half tables again: otherwise the compiler
        // keeps the first product's table values live in registers for the
        // second (at Ng = 16 that alone pushed the kernel to one wave per SIMD).
        if constexpr (FENCE || FENCE32) asm volatile("" ::: "memory");
#pragma unroll
        for (int m = 0; m < NG; ++m) x[m] = V2[c * S + m * P + p];   // column (a = p)
        line_deriv<NG>(x, z, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NG; ++b) V1[c * S + b * P + p] = z[b];
    }
    __syncthreads();

    // metric step on Gauss column (ca,cb)
    if (col) {
        const int o = cb * P + ca;
        TC ut[NG], qt[NG], wt[NG], vt[NG];
#pragma unroll
        for (int c = 0; c < NG; ++c) ut[c] = V2[c * S + o];
        line_deriv<NG>(ut, qt, Dp, Dm);
        if constexpr (FENCE || FENCE32) asm volatile("" ::: "memory");
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            // one slab at a time: without the barrier the scheduler hoists the
            // later slabs' loads and LDS reads and holds them all in registers
            if constexpr (FENCE || FENCE32) __builtin_amdgcn_sched_barrier(0);
            if (c + GPRE < NG) gload(c + GPRE);
            const TC qr = V0[c * S + o], qs = V1[c * S + o];
            const TC grr = to_compute(g[0][c], TC{}), grs = to_compute(g[1][c], TC{}),
                     grt = to_compute(g[2][c], TC{}), gss = to_compute(g[3][c], TC{}),
                     gst = to_compute(g[4][c], TC{}), gtt = to_compute(g[5][c], TC{});
            V0[c * S + o] = grr * qr + grs * qs + grt * qt[c];
            V1[c * S + o] = grs * qr + gss * qs + gst * qt[c];
            wt[c] = grt * qr + gst * qs + gtt * qt[c];
        }
        if constexpr (FENCE || FENCE32) asm volatile("" ::: "memory");
        line_deriv_t<NG>(wt, vt, Dp, Dm);
        if (lambda != TC(0)) {
            // u~ is read again from this lane's own column of V2 instead of
            // being kept live through the metric step (measured: fewer registers
            // and faster for Nq <= 10 and with LDS tables; slower at Nq = 11, 12)
            constexpr bool REREAD = TLDS || NQ <= 10;
            const int64_t wb = e * NPG;
#pragma unroll
            for (int c = 0; c < NG; ++c)
                vt[c] += lambda * ld<TC>(wJ, wb + geo_offset(ca + NG * cb, c, NG, W)) *
                         (REREAD ? V2[c * S + o] : ut[c]);
        }
#pragma unroll
        for (int c = 0; c < NG; ++c) V2[c * S + o] = vt[c];
    }
    __syncthreads();

    // s-transpose: lines (a,c) of WS, in place
    if (L < NCG) {
        const int a = L % NG, c = L / NG;
        TC v[NG], w[NG];
#pragma unroll
        for (int b = 0; b < NG; ++b) v[b] = V1[c * S + b * P + a];
        line_deriv_t<NG>(v, w, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NG; ++b) V1[c * S + b * P + a] = w[b];
    }
    // the old y column of lane (i,j) when beta != 0, requested early
    TC yold[NQ];
    if (beta != TC(0) && gll) {
        const int64_t base = e * NP + L;
#pragma unroll
        for (int k = 0; k < NQ; ++k) yold[k] = static_cast<TC>(y[base + k * NC]);
    }
    __syncthreads();

    {
        TC rIe[TLDS ? 1 : HG][HQ], rIo[TLDS ? 1 : GE][QEC];
        if constexpr (!TLDS) interp_half_tables<NQ>(I1d, rIe, rIo);
        const TC(*Ie)[HQ] = TLDS ? sIe : rIe;
        const TC(*Io)[QEC] = TLDS ? sIo : rIo;
        // r-transpose and the sum of the three terms, then r-projection: lines (b,c) -> V2 = X[c][b][i]
        if (L < NCG) {
            const int b = L % NG, c = L / NG;
            TC v[NG], w[NG], x[NQ];
#pragma unroll
            for (int a = 0; a < NG; ++a) v[a] = V0[c * S + b * P + a];
            line_deriv_t<NG>(v, w, Dp, Dm);
#pragma unroll
            for (int a = 0; a < NG; ++a) w[a] += V2[c * S + b * P + a] + V1[c * S + b * P + a];
            line_project<NQ>(w, x, Ie, Io);
#pragma unroll
            for (int i = 0; i < NQ; ++i) V2[c * S + b * P + i] = x[i];
        }
        __syncthreads();
        // s-projection: lines (i,c) -> V0 = Y[c][j][i]
        if (L < NQ * NG) {
            const int i = L % NQ, c = L / NQ;
            TC v[NG], w[NQ];
#pragma unroll
            for (int b = 0; b < NG; ++b) v[b] = V2[c * S + b * P + i];
            line_project<NQ>(v, w, Ie, Io);
#pragma unroll
            for (int j = 0; j < NQ; ++j) V0[c * S + j * P + i] = w[j];
        }
        __syncthreads();
        // t-projection: lanes (i,j) -> y[k][j][i]
        if (gll) {
            TC v[NG], w[NQ];
#pragma unroll
            for (int c = 0; c < NG; ++c) v[c] = V0[c * S + lj * P + li];
            line_project<NQ>(v, w, Ie, Io);
            const int64_t base = e * NP + L;
#pragma unroll
            for (int k = 0; k < NQ; ++k) {
                TC r = w[k] * oscale;
                if (beta != TC(0)) r += beta * yold[k];
                y[base + k * NC] = static_cast<TY>(r);
            }
        }
    }
}

}  // namespace fem

#include "bp30t2.hpp"

namespace fem {

template <int NQ, class TG, class TV>
hipError_t bp30t_launch_t(const ApplyArgs &a, hipStream_t s)
{
    using TC = typename compute_pair<TG, TV>::type;
    using TY = typename output_of<TV>::type;
    if (a.E < 1) return hipSuccess;
    const TC oscale = static_cast<TC>(is_f16_prec(a.prec) ? a.out_scale / a.geo_scale
                                                                         : a.out_scale);
    // one workgroup per element; a grid cap splits the elements over launches
    int64_t chunk = a.grid_cap > 0 ? a.grid_cap : a.E;
    if (chunk > max_grid(bp30t_threads(NQ))) chunk = max_grid(bp30t_threads(NQ));
    for (int64_t e0 = 0; e0 < a.E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(a.E - e0 < chunk ? a.E - e0 : chunk);
        if constexpr (bp30t_two_volumes(NQ, sizeof(TC)))
            hipLaunchKernelGGL((bp30t2_kernel<NQ, TG, TV>), dim3(grid), dim3(bp30t_threads(NQ)), 0, s, a.E, a.I1d,
                               a.Dgl, static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                               static_cast<TC>(a.lambda), static_cast<const TV *>(a.u), static_cast<TY *>(a.y),
                               static_cast<TC>(a.beta), oscale, e0);
        else
            hipLaunchKernelGGL((bp30t_kernel<NQ, TG, TV>), dim3(grid), dim3(bp30t_threads(NQ)), 0, s, a.E, a.I1d,
                               a.Dgl, static_cast<const TG *>(a.G), static_cast<const TG *>(a.wJ),
                               static_cast<TC>(a.lambda), static_cast<const TV *>(a.u), static_cast<TY *>(a.y),
                               static_cast<TC>(a.beta), oscale, e0);
    }
    return hipGetLastError();
}

}  // namespace fem
