// bp30t2.hpp -- BP3.0 de-aliased stiffness (Alg. 5 with the interpolation and
// projection of Alg. 1-2), line per lane as in bp30t.hpp, with two Ng^3 LDS
// volumes instead of three.  For FP64 arithmetic at high degree: at Ng = 12 and
// from Ng = 14 the third volume took the LDS a second workgroup needs, so each
// CU held one element at a time and its HBM traffic stalled at every barrier.
//
// Every turn between line directions works in place where the line's lane
// owns all the locations it reads and writes, and the metric lane keeps the
// t-direction in registers across the phases that need a third volume:
//   t-interpolation   lanes (i,j): u column                  -> V0 = A[c][j][i]
//   s-interpolation   lines (i,c), in place in V0           -> B[c][b][i]
//   r-interpolation   lines (b,c): B row -> u~ row           -> V1 = U[c][b][a]
//     + r-derivative  of the same row, in place in V0        -> QR
//   (column read)     lane (a,b) keeps its u~ column in registers
//   s-derivative      lines (a,c), in place in V1            -> QS
//   metric            columns (a,b): qt = D~ u~ (registers); WR over QR, WS
//                     over QS; v = D~^T wt + lambda wJ u~ kept in registers
//   s-transpose       lines (a,c), in place in V1            -> D~^T WS
//   (column add)      lane (a,b) adds v into V1
//   r-transpose       lines (b,c): D~^T WR row + V1 row, r-projected, in place in V0
//   s-projection      lines (i,c), in place in V0            -> Y[c][j][i]
//   t-projection      lanes (i,j)                            -> y[k][j][i]
// Every sum is taken in the order bp30t_kernel takes it, so the two kernels
// give the same bits.  Half tables live in LDS; an empty asm with a memory
// clobber between consecutive line products keeps the compiler from holding
// one product's table values in registers for the next.
// Included by bp30t.hpp (after bp30t_threads), whose launcher picks the kernel.
#pragma once

#include "bp35.hpp"
#include "lines.hpp"

namespace fem {

// Slabs of factors requested ahead of their use in the metric step: two; one
// at Ng = 17.  There, asking the register allocator for three waves per SIMD
// (two five-wave workgroups per CU) measured 2% faster but spilled 120 bytes
// per lane, which went to HBM as scratch traffic; the kernel runs without.
// At Nq = 12 the request (172 -> 168 VGPRs, 28 bytes of spill) lets four
// workgroups share a CU instead of two: 4.05 -> 3.87 ms at E = 131072, against
// 4.15 ms for the three-volume kernel, with the same bits.
constexpr int bp30t2_gpre(int nq) { return nq >= 16 ? 1 : 2; }
constexpr int bp30t2_min_waves(int nq) { return nq == 12 ? 3 : 1; }

template <int NQ, class TG, class TV>
__global__ __launch_bounds__(bp30t_threads(NQ))
__attribute__((amdgpu_waves_per_eu(bp30t2_min_waves(NQ)))) void bp30t2_kernel(
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
    constexpr int P = lds_row(NG, sizeof(TC));
    constexpr int S = NG * P;
    constexpr int VOL = NG * S;
    constexpr int W = geo_vec(NG, sizeof(TG));
    constexpr int QEC = QE > 0 ? QE : 1;
    constexpr int GPRE = bp30t2_gpre(NQ);
    static_assert(NCG <= bp30t_threads(NQ), "one lane per Gauss column");

    __shared__ __align__(16) TC V0[VOL];
    __shared__ __align__(16) TC V1[VOL];
    __shared__ TC sIe[HG][HQ];
    __shared__ TC sIo[GE][QEC];
    __shared__ TC sDp[GE][HG];
    __shared__ TC sDm[HG][GE];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;
    const bool col = L < NCG;                    // owns Gauss column (ca, cb)
    const int ca = L % NG, cb = L / NG;
    const bool gll = L < NC;                     // owns GLL column (li, lj)
    const int li = L % NQ, lj = L / NQ;

    // requests, oldest first: the lane's table entries, its u column, the
    // first GPRE slabs of its Gauss column's factors (every lane issues them;
    // lanes without a column re-read another column and never use it)
    double ti0, ti1, td0, td1;
    interp_pair_load<NQ>(I1d, L, ti0, ti1);
    deriv_pair_load<NG>(Dgl, L, td0, td1);
    __builtin_amdgcn_sched_barrier(0);
    TV uraw[NQ];
    {
        const int64_t base = e * NP + (gll ? L : 0);
#pragma unroll
        for (int k = 0; k < NQ; ++k) uraw[k] = u[base + k * NC];
    }
    __builtin_amdgcn_sched_barrier(0);
    TG g[6][NG];
    const int64_t gb = e * (6 * NPG);
    const int gcol = col ? L : (L & ~(kWave - 1));   // as in bp30t_kernel
    auto gload = [&](int c) {
#pragma unroll
        for (int f = 0; f < 6; ++f) g[f][c] = nt_load(G + gb + f * NPG + geo_offset(gcol, c, NG, W));
    };
#pragma unroll
    for (int c = 0; c < GPRE; ++c) gload(c);
    __builtin_amdgcn_sched_barrier(0);
    interp_pair_store<NQ>(sIe, sIo, L, ti0, ti1);
    deriv_pair_store<NG>(sDp, sDm, L, td0, td1);
    __syncthreads();
    TC uc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        uc[k] = to_compute(uraw[k], TC{});
        asm volatile("" : "+v"(uc[k]));   // keeps the u loads out of the branch below
    }

    // t-interpolation: lanes (i,j) -> V0 = A[c][j][i]
    if (gll) {
        TC z[NG];
        line_interp<NQ>(uc, z, sIe, sIo);
#pragma unroll
        for (int c = 0; c < NG; ++c) V0[c * S + lj * P + li] = z[c];
    }
    __syncthreads();
    // s-interpolation, in place: lines (i,c) of V0 -> B[c][b][i]
    if (L < NQ * NG) {
        const int i = L % NQ, c = L / NQ;
        TC x[NQ], z[NG];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[c * S + m * P + i];
        line_interp<NQ>(x, z, sIe, sIo);
#pragma unroll
        for (int b = 0; b < NG; ++b) V0[c * S + b * P + i] = z[b];
    }
    __syncthreads();
    // r-interpolation: lines (b,c): u~ row -> V1; its r-derivative in place in V0
    if (L < NCG) {
        const int b = L % NG, c = L / NG;
        TC x[NQ], z[NG], q[NG];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[c * S + b * P + m];
        line_interp<NQ>(x, z, sIe, sIo);
#pragma unroll
        for (int a = 0; a < NG; ++a) V1[c * S + b * P + a] = z[a];
        asm volatile("" ::: "memory");
        line_deriv<NG>(z, q, sDp, sDm);
#pragma unroll
        for (int a = 0; a < NG; ++a) V0[c * S + b * P + a] = q[a];
    }
    __syncthreads();
    // the metric lane's u~ column, read before the s-derivative overwrites it
    const int o = cb * P + ca;
    TC ut[NG];
    if (col) {
#pragma unroll
        for (int c = 0; c < NG; ++c) ut[c] = V1[c * S + o];
    }
    __syncthreads();
    // s-derivative, in place: lines (a,c) of V1 -> QS
    if (L < NCG) {
        const int a = L % NG, c = L / NG;
        TC x[NG], z[NG];
#pragma unroll
        for (int m = 0; m < NG; ++m) x[m] = V1[c * S + m * P + a];
        line_deriv<NG>(x, z, sDp, sDm);
#pragma unroll
        for (int b = 0; b < NG; ++b) V1[c * S + b * P + a] = z[b];
    }
    __syncthreads();

    // metric step on Gauss column (ca,cb)
    TC vt[NG];
    if (col) {
        TC qt[NG], wt[NG];
        asm volatile("" ::: "memory");
        line_deriv<NG>(ut, qt, sDp, sDm);
        asm volatile("" ::: "memory");
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            // one slab at a time (the scheduler would otherwise hoist the later
            // slabs' loads and LDS reads and hold them all in registers)
            __builtin_amdgcn_sched_barrier(0);
            if (c + GPRE < NG) gload(c + GPRE);
            const TC qr = V0[c * S + o], qs = V1[c * S + o];
            const TC grr = to_compute(g[0][c], TC{}), grs = to_compute(g[1][c], TC{}),
                     grt = to_compute(g[2][c], TC{}), gss = to_compute(g[3][c], TC{}),
                     gst = to_compute(g[4][c], TC{}), gtt = to_compute(g[5][c], TC{});
            V0[c * S + o] = grr * qr + grs * qs + grt * qt[c];
            V1[c * S + o] = grs * qr + gss * qs + gst * qt[c];
            wt[c] = grt * qr + gst * qs + gtt * qt[c];
        }
        asm volatile("" ::: "memory");
        line_deriv_t<NG>(wt, vt, sDp, sDm);
        if (lambda != TC(0)) {
            const int64_t wb = e * NPG;
#pragma unroll
            for (int c = 0; c < NG; ++c)
                vt[c] += lambda * ld<TC>(wJ, wb + geo_offset(ca + NG * cb, c, NG, W)) * ut[c];
        }
    }
    __syncthreads();
    // s-transpose, in place: lines (a,c) of WS
    if (L < NCG) {
        const int a = L % NG, c = L / NG;
        TC v[NG], w[NG];
#pragma unroll
        for (int b = 0; b < NG; ++b) v[b] = V1[c * S + b * P + a];
        line_deriv_t<NG>(v, w, sDp, sDm);
#pragma unroll
        for (int b = 0; b < NG; ++b) V1[c * S + b * P + a] = w[b];
    }
    __syncthreads();
    // the t-term joins the s-term (vt + D~^T WS, the order bp30t_kernel sums in)
    if (col) {
#pragma unroll
        for (int c = 0; c < NG; ++c) V1[c * S + o] = vt[c] + V1[c * S + o];
    }
    __syncthreads();
    // r-transpose, the sum of the three terms, r-projection: lines (b,c), in place in V0
    if (L < NCG) {
        const int b = L % NG, c = L / NG;
        TC v[NG], w[NG], x[NQ];
#pragma unroll
        for (int a = 0; a < NG; ++a) v[a] = V0[c * S + b * P + a];
        line_deriv_t<NG>(v, w, sDp, sDm);
#pragma unroll
        for (int a = 0; a < NG; ++a) w[a] += V1[c * S + b * P + a];
        asm volatile("" ::: "memory");
        line_project<NQ>(w, x, sIe, sIo);
#pragma unroll
        for (int i = 0; i < NQ; ++i) V0[c * S + b * P + i] = x[i];
    }
    __syncthreads();
    // s-projection, in place: lines (i,c) -> Y[c][j][i]
    if (L < NQ * NG) {
        const int i = L % NQ, c = L / NQ;
        TC v[NG], w[NQ];
#pragma unroll
        for (int b = 0; b < NG; ++b) v[b] = V0[c * S + b * P + i];
        line_project<NQ>(v, w, sIe, sIo);
#pragma unroll
        for (int j = 0; j < NQ; ++j) V0[c * S + j * P + i] = w[j];
    }
    __syncthreads();
    // t-projection: lanes (i,j) -> y[k][j][i]
    if (gll) {
        const int64_t base = e * NP + L;
        TC v[NG], w[NQ], yold[NQ];
        if (beta != TC(0)) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) yold[k] = static_cast<TC>(y[base + k * NC]);
        }
#pragma unroll
        for (int c = 0; c < NG; ++c) v[c] = V0[c * S + lj * P + li];
        line_project<NQ>(v, w, sIe, sIo);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            TC r = w[k] * oscale;
            if (beta != TC(0)) r += beta * yold[k];
            y[base + k * NC] = static_cast<TY>(r);
        }
    }
}

}  // namespace fem
