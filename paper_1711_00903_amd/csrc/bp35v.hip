// bp35v.hip -- BP3.5 collocated stiffness (Alg. 4), FP64, with the geometric
// factors of every GLL point evaluated inside the kernel from the element's
// 8 vertices (the trilinear map of the Problem description section) instead of
// read from memory.  The BP3.5 optimisation section notes that the factors
// could be computed on the fly from the vertices and loads them instead; on
// gfx950, whose FP64 rate per byte of HBM is several times that of the GPU
// the paper used, the trade is worth re-measuring: a point then moves 16 B of
// fields instead of 64 B, for about 50 extra FMAs and one division.
//
// Line-per-lane structure of bp35t.hpp (one element per workgroup, two LDS
// volumes, derivative half tables in LDS).  The metric step of column (i,j)
// forms, at t = t_k, the covariant vectors
//   a_r = A0 + t A1,  a_s = B0 + t B1,  a_t = C
// (a_r and a_s are linear in t along a column, a_t constant), the cross
// products c_r = a_s x a_t, c_s = a_t x a_r, c_t = a_r x a_s, |J| = a_r . c_r,
// and G_ab = w_i w_j w_k (c_a . c_b) / |J|, the same factors the set-up kernel
// writes (geometry.hip), up to rounding.
#include "fem_device.hpp"
#include "launch.hpp"
#include "lines.hpp"
#include "tiles.hpp"

namespace fem {

struct GllRule {
    double r[kMaxN + 1];
    double w[kMaxN + 1];
};

constexpr int bp35v_threads(int nq) { return round_up_wave(nq * nq); }

// Waves per SIMD asked of the register allocator: three up to Nq = 6, where
// that spills nothing (N = 5: +7%); at Nq = 7, 8 it would spill and was slower.
constexpr int bp35v_min_waves(int nq) { return nq <= 6 ? 3 : 1; }

template <int NQ>
__global__ __launch_bounds__(bp35v_threads(NQ))
__attribute__((amdgpu_waves_per_eu(bp35v_min_waves(NQ)))) void bp35v_kernel(const double *__restrict__ D1d,
                                                                  const double *__restrict__ X, GllRule rule,
                                                                  double lambda, const double *__restrict__ u,
                                                                  double *__restrict__ y, double beta, int64_t e0)
{
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int HQ = (NQ + 1) / 2, QE = NQ / 2;
    constexpr int P = lds_row(NQ, 8);
    constexpr int S = NQ * P;
    constexpr int VOL = NQ * S;
    static_assert(NQ >= 2 && NC <= bp35v_threads(NQ), "one lane per GLL column");

    __shared__ __align__(16) double V0[VOL];
    __shared__ __align__(16) double V1[VOL];
    __shared__ double sDp[QE][HQ];
    __shared__ double sDm[HQ][QE];

    const int L = threadIdx.x;
    const int64_t e = e0 + blockIdx.x;
    const bool own = L < NC;          // owns column (ci,cj) and lines (lp, lk)
    const int gcol = own ? L : 0;     // lanes beyond re-read column 0 and never store
    const int ci = gcol % NQ, cj = gcol / NQ;
    const int lp = ci, lk = cj;

    // requests, oldest first: this lane's pair of table entries, then the u
    // column (every lane loads, so the compiler counts the requests in flight)
    double td0, td1;
    deriv_pair_load<NQ>(D1d, L, td0, td1);
    __builtin_amdgcn_sched_barrier(0);
    double uc[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) uc[k] = u[e * NP + gcol + k * NC];
    __builtin_amdgcn_sched_barrier(0);

    // the column's covariant-vector coefficients, formed before the first
    // barrier (the element's vertices are uniform: scalar loads); the column's
    // reference coordinates and weights by selects (no dynamic indexing of the
    // argument block)
    double r = 0.0, s = 0.0, wi = 0.0, wj = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        r = ci == q ? rule.r[q] : r;
        wi = ci == q ? rule.w[q] : wi;
        s = cj == q ? rule.r[q] : s;
        wj = cj == q ? rule.w[q] : wj;
    }
    // vertex v = a + 2b + 4c at reference corner (2a-1, 2b-1, 2c-1)
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

    const double wij = wi * wj;
    deriv_pair_store<NQ>(sDp, sDm, L, td0, td1);
    if (own) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) V0[k * S + cj * P + ci] = uc[k];
    }
    __syncthreads();
    const double(*Dp)[HQ] = sDp;
    const double(*Dm)[QE] = sDm;

    // r-derivative: row (j = lp) of slab lk -> V1
    if (own) {
        double x[NQ], z[NQ];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[lk * S + lp * P + m];
        line_deriv<NQ>(x, z, Dp, Dm);
#pragma unroll
        for (int a = 0; a < NQ; ++a) V1[lk * S + lp * P + a] = z[a];
    }
    __syncthreads();
    // s-derivative: column (i = lp) of slab lk, in place in V0
    if (own) {
        double x[NQ], z[NQ];
#pragma unroll
        for (int m = 0; m < NQ; ++m) x[m] = V0[lk * S + m * P + lp];
        line_deriv<NQ>(x, z, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NQ; ++b) V0[lk * S + b * P + lp] = z[b];
    }
    __syncthreads();

    // metric step on column (ci,cj), with the factors formed here
    double vt[NQ];
    if (own) {
        const int o = cj * P + ci;
        double qt[NQ], wt[NQ], wdet[NQ];
        line_deriv<NQ>(uc, qt, Dp, Dm);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double t = rule.r[k];
            const double ar[3] = {A0[0] + t * A1[0], A0[1] + t * A1[1], A0[2] + t * A1[2]};
            const double as[3] = {B0[0] + t * B1[0], B0[1] + t * B1[1], B0[2] + t * B1[2]};
            const double cr[3] = {as[1] * C[2] - as[2] * C[1], as[2] * C[0] - as[0] * C[2],
                                  as[0] * C[1] - as[1] * C[0]};
            const double cs[3] = {C[1] * ar[2] - C[2] * ar[1], C[2] * ar[0] - C[0] * ar[2],
                                  C[0] * ar[1] - C[1] * ar[0]};
            const double ct[3] = {ar[1] * as[2] - ar[2] * as[1], ar[2] * as[0] - ar[0] * as[2],
                                  ar[0] * as[1] - ar[1] * as[0]};
            const double det = ar[0] * cr[0] + ar[1] * cr[1] + ar[2] * cr[2];
            const double w = wij * rule.w[k];
            wdet[k] = w * det;
            const double f = w / det;
            const double grr = f * (cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
            const double grs = f * (cr[0] * cs[0] + cr[1] * cs[1] + cr[2] * cs[2]);
            const double grt = f * (cr[0] * ct[0] + cr[1] * ct[1] + cr[2] * ct[2]);
            const double gss = f * (cs[0] * cs[0] + cs[1] * cs[1] + cs[2] * cs[2]);
            const double gst = f * (cs[0] * ct[0] + cs[1] * ct[1] + cs[2] * ct[2]);
            const double gtt = f * (ct[0] * ct[0] + ct[1] * ct[1] + ct[2] * ct[2]);
            const double qr = V1[k * S + o], qs = V0[k * S + o];
            V1[k * S + o] = grr * qr + grs * qs + grt * qt[k];
            V0[k * S + o] = grs * qr + gss * qs + gst * qt[k];
            wt[k] = grt * qr + gst * qs + gtt * qt[k];
        }
        line_deriv_t<NQ>(wt, vt, Dp, Dm);
        if (lambda != 0.0) {
#pragma unroll
            for (int k = 0; k < NQ; ++k) vt[k] += lambda * wdet[k] * uc[k];
        }
    }
    // the old y column when beta != 0, requested before the transposes
    double yold[NQ];
    if (beta != 0.0 && own) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) yold[k] = y[e * NP + L + k * NC];
    }
    __syncthreads();

    // transposes, in place: s-line (lp,lk) of WS and r-line (lp,lk) of WR
    if (own) {
        double v[NQ], w[NQ];
#pragma unroll
        for (int b = 0; b < NQ; ++b) v[b] = V0[lk * S + b * P + lp];
        line_deriv_t<NQ>(v, w, Dp, Dm);
#pragma unroll
        for (int b = 0; b < NQ; ++b) V0[lk * S + b * P + lp] = w[b];
#pragma unroll
        for (int a = 0; a < NQ; ++a) v[a] = V1[lk * S + lp * P + a];
        line_deriv_t<NQ>(v, w, Dp, Dm);
#pragma unroll
        for (int a = 0; a < NQ; ++a) V1[lk * S + lp * P + a] = w[a];
    }
    __syncthreads();

    if (own) {
        const int o = cj * P + ci;
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            double r = V0[k * S + o] + V1[k * S + o] + vt[k];
            if (beta != 0.0) r += beta * yold[k];
            y[e * NP + L + k * NC] = r;
        }
    }
}

template <int NQ>
static hipError_t bp35v_launch_t(int64_t E, const double *D1d, const double *X, const GllRule &rule,
                                 double lambda, const double *u, double *y, double beta, int64_t grid_cap,
                                 hipStream_t s)
{
    // one workgroup per element; a grid cap splits the elements over launches
    int64_t chunk = grid_cap > 0 ? grid_cap : E;
    if (chunk > max_grid(bp35v_threads(NQ))) chunk = max_grid(bp35v_threads(NQ));
    for (int64_t e0 = 0; e0 < E; e0 += chunk) {
        const unsigned grid = static_cast<unsigned>(E - e0 < chunk ? E - e0 : chunk);
        hipLaunchKernelGGL((bp35v_kernel<NQ>), dim3(grid), dim3(bp35v_threads(NQ)), 0, s, D1d, X, rule, lambda,
                           u, y, beta, e0);
    }
    return hipGetLastError();
}

hipError_t launch_bp35v(int N, int64_t E, const double *D1d, const double *X, double lambda, const double *u,
                        double *y, double beta, int64_t grid_cap, hipStream_t s)
{
    if (E < 1) return hipSuccess;
    GllRule rule{};
    if (gauss_lobatto(N, rule.r, rule.w)) return hipErrorInvalidValue;
    switch (N + 1) {
    case 2: return bp35v_launch_t<2>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 3: return bp35v_launch_t<3>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 4: return bp35v_launch_t<4>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 5: return bp35v_launch_t<5>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 6: return bp35v_launch_t<6>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 7: return bp35v_launch_t<7>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 8: return bp35v_launch_t<8>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 9: return bp35v_launch_t<9>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 10: return bp35v_launch_t<10>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 11: return bp35v_launch_t<11>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 12: return bp35v_launch_t<12>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 13: return bp35v_launch_t<13>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 14: return bp35v_launch_t<14>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 15: return bp35v_launch_t<15>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    case 16: return bp35v_launch_t<16>(E, D1d, X, rule, lambda, u, y, beta, grid_cap, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace fem
