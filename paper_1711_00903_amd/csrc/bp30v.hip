// bp30v.hip -- BP3.0 de-aliased stiffness (Alg. 5), FP64, with the geometric
// factors of every Gauss point evaluated inside the kernel from the element's
// 8 vertices (the trilinear map of the Problem description section) instead
// of read from memory: the trade the BP3.5 optimisation section weighs, here
// for the operator whose factors dominate its traffic (6 Ng^3 values per
// element, 81% of the bytes at N = 7).  A GLL point then moves 16 B of
// fields.  The kernel is the line-per-lane BP3.0 kernel (bp30t.hpp) with the
// factor loads replaced by the metric computation of bp35v.hip at the Gauss
// points.
#include "fem_device.hpp"
#include "launch.hpp"
#include "lines.hpp"
#include "tiles.hpp"

namespace fem {

struct GlRule {
    double r[kMaxN + 2];
    double w[kMaxN + 2];
};

constexpr int bp30v_threads(int nq) { return round_up_wave((nq + 1) * (nq + 1)); }

template <int NQ, class TG, class TV>
__global__ __launch_bounds__(bp30v_threads(NQ)) void bp30v_kernel(
    int64_t E, const double *__restrict__ I1d, const double *__restrict__ Dgl, const double *__restrict__ X,
    GlRule rule, typename compute_pair<TG, TV>::type lambda, const TV *__restrict__ u,
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
    static_assert(NCG <= bp30v_threads(NQ), "one lane per Gauss column");

    __shared__ __align__(16) TC V0[VOL];
    __shared__ __align__(16) TC V1[VOL];
    __shared__ __align__(16) TC V2[VOL];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;
    const bool col = L < NCG;                    // owns Gauss column (ca, cb)
    const int ca = L % NG, cb = L / NG;

    // the u column of lane (i,j) and the 6 Ng factors of Gauss column (ca,cb).
    // Every lane loads (lanes beyond the columns re-read column 0 and never use
    // it): under a lane condition the compiler widens a narrow value inside the
    // branch and waits for it there, one load at a time.  The u column is
    // requested first and waited for only after the factor requests are out.
    const bool gll = L < NC;
    const int li = L % NQ, lj = L / NQ;
    // Half tables: in registers for small Nq, in LDS beyond (the lines then
    // need the registers); the LDS copies are fetched ahead of the element's
    // loads and stored once those are issued.  The crossover was measured at
    // E = 262144: LDS from Nq = 11 (Nq = 12 in FP64 arithmetic stays faster
    // with registers).
    constexpr bool TLDS = NQ > 12 || NQ == 11 || (NQ == 12 && sizeof(TC) == 4);
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
    // the column's covariant-vector coefficients at Gauss point (ca,cb): a_r and
    // a_s linear in t, a_t constant along the column (the element's vertices
    // are uniform: scalar loads); coordinates and weights by selects
    const int gcol = col ? L : 0;
    const int ga = gcol % NG, gb = gcol / NG;
    double r = 0.0, s = 0.0, wa = 0.0, wb = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        r = ga == q ? rule.r[q] : r;
        wa = ga == q ? rule.w[q] : wa;
        s = gb == q ? rule.r[q] : s;
        wb = gb == q ? rule.w[q] : wb;
    }
    const double *Xe = X + 24 * e;
    double A0[3] = {0, 0, 0}, A1[3] = {0, 0, 0}, B0[3] = {0, 0, 0}, B1[3] = {0, 0, 0}, C[3] = {0, 0, 0};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double xi = (v & 1) ? 1.0 : -1.0, eta = (v & 2) ? 1.0 : -1.0, zeta = (v & 4) ? 1.0 : -1.0;
        const double fr = 0.125 * xi * (1.0 + eta * s);
        const double fs = 0.125 * eta * (1.0 + xi * r);
        const double ft = 0.125 * zeta * (1.0 + xi * r) * (1.0 + eta * s);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double p = Xe[3 * v + d];
            A0[d] += fr * p;
            A1[d] += fr * zeta * p;
            B0[d] += fs * p;
            B1[d] += fs * zeta * p;
            C[d] += ft * p;
        }
    }
    const double wab = wa * wb;
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
        TC ut[NG], qt[NG], wt[NG], vt[NG], wdet[NG];
#pragma unroll
        for (int c = 0; c < NG; ++c) ut[c] = V2[c * S + o];
        line_deriv<NG>(ut, qt, Dp, Dm);
#pragma unroll
        for (int c = 0; c < NG; ++c) {
            const double t = rule.r[c];
            const double ar[3] = {A0[0] + t * A1[0], A0[1] + t * A1[1], A0[2] + t * A1[2]};
            const double as[3] = {B0[0] + t * B1[0], B0[1] + t * B1[1], B0[2] + t * B1[2]};
            const double cr[3] = {as[1] * C[2] - as[2] * C[1], as[2] * C[0] - as[0] * C[2],
                                  as[0] * C[1] - as[1] * C[0]};
            const double cs[3] = {C[1] * ar[2] - C[2] * ar[1], C[2] * ar[0] - C[0] * ar[2],
                                  C[0] * ar[1] - C[1] * ar[0]};
            const double ct[3] = {ar[1] * as[2] - ar[2] * as[1], ar[2] * as[0] - ar[0] * as[2],
                                  ar[0] * as[1] - ar[1] * as[0]};
            const double det = ar[0] * cr[0] + ar[1] * cr[1] + ar[2] * cr[2];
            const double w = wab * rule.w[c];
            wdet[c] = w * det;
            const double f = w / det;
            const TC qr = V0[c * S + o], qs = V1[c * S + o];
            const TC grr = f * (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            const TC grs = f * (cr[0] * cs[0] + cr[1] * cs[1] + cr[2] * cs[2]);
            const TC grt = f * (cr[0] * ct[0] + cr[1] * ct[1] + cr[2] * ct[2]);
            const TC gss = f * (cs[0] * cs[0] + cs[1] * cs[1] + cs[2] * cs[2]);
            const TC gst = f * (cs[0] * ct[0] + cs[1] * ct[1] + cs[2] * ct[2]);
            const TC gtt = f * (ct[0] * ct[0] + ct[1] * ct[1] + ct[2] * ct[2]);
            V0[c * S + o] = grr * qr + grs * qs + grt * qt[c];
            V1[c * S + o] = grs * qr + gss * qs + gst * qt[c];
            wt[c] = grt * qr + gst * qs + gtt * qt[c];
        }
        line_deriv_t<NG>(wt, vt, Dp, Dm);
        if (lambda != TC(0)) {
#pragma unroll
            for (int c = 0; c < NG; ++c) vt[c] += lambda * wdet[c] * V2[c * S + o];
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

template <int NQ>
static hipError_t bp30v_launch_t(int64_t E, const double *I1d, const double *Dgl, const double *X,
                                 const GlRule &rule, double lambda, const double *u, double *y, double beta,
                                 hipStream_t s)
{
    // one workgroup per element, split over launches of at most max_grid workgroups
    const int64_t chunk = max_grid(bp30v_threads(NQ));
    for (int64_t e0 = 0; e0 < E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(E - e0 < chunk ? E - e0 : chunk);
        hipLaunchKernelGGL((bp30v_kernel<NQ, double, double>), dim3(grid), dim3(bp30v_threads(NQ)), 0, s, E, I1d,
                           Dgl, X, rule, lambda, u, y, beta, 1.0, e0);
    }
    return hipGetLastError();
}

hipError_t launch_bp30v(int N, int64_t E, const double *I1d, const double *Dgl, const double *X, double lambda,
                        const double *u, double *y, double beta, hipStream_t s)
{
    if (E < 1) return hipSuccess;
    GlRule rule{};
    if (gauss_legendre(N + 2, rule.r, rule.w)) return hipErrorInvalidValue;
    switch (N + 1) {
    case 2: return bp30v_launch_t<2>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 3: return bp30v_launch_t<3>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 4: return bp30v_launch_t<4>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 5: return bp30v_launch_t<5>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 6: return bp30v_launch_t<6>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 7: return bp30v_launch_t<7>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 8: return bp30v_launch_t<8>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 9: return bp30v_launch_t<9>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 10: return bp30v_launch_t<10>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 11: return bp30v_launch_t<11>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 12: return bp30v_launch_t<12>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 13: return bp30v_launch_t<13>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 14: return bp30v_launch_t<14>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 15: return bp30v_launch_t<15>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    case 16: return bp30v_launch_t<16>(E, I1d, Dgl, X, rule, lambda, u, y, beta, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
