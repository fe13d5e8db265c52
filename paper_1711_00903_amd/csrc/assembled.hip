// assembled.hip -- the assembled (continuous) screened-Poisson operator
// Z^T (S + lambda M) Z of a conforming hex mesh, its diagonal, and
// Jacobi-preconditioned conjugate gradients on it.
//
// The paper applies the element matrices as one block-diagonal operator, each
// element on its own copy of its nodes (Problem description section).  The
// global finite-element operator sums the same blocks into the nodes that
// neighbouring elements share: with Z the Boolean gather from global to
// element-local nodes, A = Z^T A_L Z.  Here
//   * Z is an index gather (ul[l] = ug[gather[l]]);
//   * Z^T sums each global node's local copies through a compressed
//     inverse map (offsets / locals, the local copies in ascending order), so
//     every sum is taken in one fixed order: no atomics, bitwise repeatable;
//   * A_L is the library's BP3.5 stiffness plus lambda times the BP1.0 mass
//     (the operator of fem_cg_solve), applied by the element kernels.
// Index maps come from the caller; every index is checked against its range
// before it is used (an entry out of range reads as zero), so a bad map gives
// wrong numbers, never an access outside the arrays.
//
// Jacobi preconditioner: diag(Z^T A_L Z) = Z^T diag(A_L), with the diagonal of
// one element's S + lambda M written out from the operators' definitions:
//   S_nn = sum_a D[a][i]^2 G_rr(a,j,k) + sum_b D[b][j]^2 G_ss(i,b,k)
//        + sum_c D[c][k]^2 G_tt(i,j,c)
//        + 2 (D[i][i] D[j][j] G_rs + D[i][i] D[k][k] G_rt + D[j][j] D[k][k] G_st)(n)
//   M_nn = sum_abc wJ(a,b,c) I[a][i]^2 I[b][j]^2 I[c][k]^2.
#include <chrono>
#include <cmath>

#include "fem.h"
#include "fem_device.hpp"
#include "launch.hpp"

namespace fem {

constexpr int kAsThreads = 256;
constexpr int kAsPer = 4;   // entries per thread of the chunked vector kernels
constexpr int64_t kAsChunk = static_cast<int64_t>(kAsThreads) * kAsPer;

inline int64_t as_blocks(int64_t n)
{
    const int64_t b = (n + kAsChunk - 1) / kAsChunk;
    return b > 0 ? b : 1;
}

// Sum of v over the workgroup (kAsThreads lanes), in a fixed order: within
// each wave by shuffles, then the waves in order.
__device__ __forceinline__ double wg_sum(double v)
{
    __shared__ double red[kAsThreads / kWave];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int w = 0; w < kAsThreads / kWave; ++w) s += red[w];
    return s;
}

// ul[l] = ug[gather[l]] (Z u).
__global__ __launch_bounds__(kAsThreads) void gather_kernel(const int32_t *__restrict__ gid,
                                                            const double *__restrict__ ug,
                                                            double *__restrict__ ul, int64_t nl, int64_t ng)
{
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
    int64_t g[kAsPer];
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t l = base + q * kAsThreads;
        g[q] = l < nl ? gid[l] : -1;
    }
    double v[kAsPer];
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) v[q] = (g[q] >= 0 && g[q] < ng) ? ug[g[q]] : 0.0;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t l = base + q * kAsThreads;
        if (l < nl) ul[l] = v[q];
    }
}

// ug[g] = sum of ul[locals[k]], k in [offsets[g], offsets[g+1]) (Z^T u); with
// pdot set, also per-workgroup partials of pdot[g] * ug[g] into part.
__global__ __launch_bounds__(kAsThreads) void scatter_kernel(const int32_t *__restrict__ off,
                                                             const int32_t *__restrict__ loc,
                                                             const double *__restrict__ ul,
                                                             double *__restrict__ ug, int64_t ng, int64_t nl,
                                                             const double *__restrict__ pdot,
                                                             double *__restrict__ part)
{
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
    double dot = 0.0;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g >= ng) continue;
        int64_t k0 = off[g], k1 = off[g + 1];
        k0 = k0 < 0 ? 0 : (k0 > nl ? nl : k0);
        k1 = k1 < k0 ? k0 : (k1 > nl ? nl : k1);
        double s = 0.0;
        for (int64_t k = k0; k < k1; ++k) {
            const int64_t l = loc[k];
            if (l >= 0 && l < nl) s += ul[l];
        }
        ug[g] = s;
        if (pdot) dot += pdot[g] * s;
    }
    if (part) {
        const double t = wg_sum(dot);
        if (threadIdx.x == 0) part[blockIdx.x] = t;
    }
}

// Diagonal of each element's S + lambda M (formulas above), one workgroup
// per element, one lane per GLL column (i,j).  FP64 data in the library's
// interleaved geometric layout.
template <int NQ>
__global__ __launch_bounds__(round_up_wave(NQ *NQ)) void elem_diag_kernel(
    int64_t E, const double *__restrict__ D1d, const double *__restrict__ I1d, const double *__restrict__ G,
    const double *__restrict__ wJ, double lambda, double *__restrict__ dl, int64_t e0)
{
    constexpr int NG = NQ + 1;
    constexpr int NC = NQ * NQ;
    constexpr int NP = NC * NQ;
    constexpr int NCG = NG * NG;
    constexpr int NPG = NCG * NG;
    constexpr int WG = geo_vec(NQ, 8), WW = geo_vec(NG, 8);
    __shared__ double sD2[NQ * NQ], sDd[NQ], sI2[NG * NQ], sw[NPG];
    const int64_t e = e0 + blockIdx.x;
    const int t = threadIdx.x;
    for (int q = t; q < NQ * NQ; q += blockDim.x) sD2[q] = D1d[q] * D1d[q];
    for (int q = t; q < NQ; q += blockDim.x) sDd[q] = D1d[q * NQ + q];
    for (int q = t; q < NG * NQ; q += blockDim.x) sI2[q] = I1d[q] * I1d[q];
    if (lambda != 0.0)
        for (int q = t; q < NPG; q += blockDim.x) {
            const int col = q % NCG, c = q / NCG;
            sw[q] = wJ[e * NPG + geo_offset(col, c, NG, WW)];
        }
    __syncthreads();
    if (t >= NC) return;
    const int i = t % NQ, j = t / NQ;
    const double *Ge = G + e * 6 * static_cast<int64_t>(NP);
    auto g = [&](int f, int col, int k) { return Ge[f * NP + geo_offset(col, k, NQ, WG)]; };
    // mass: T[c] = sum_b I[b][j]^2 sum_a I[a][i]^2 wJ(a,b,c), then per k the c-sum
    double T[NG];
#pragma unroll
    for (int c = 0; c < NG; ++c) {
        double sb = 0.0;
        if (lambda != 0.0)
            for (int b = 0; b < NG; ++b) {
                double sa = 0.0;
                for (int a = 0; a < NG; ++a) sa += sI2[a * NQ + i] * sw[a + NG * b + NCG * c];
                sb += sI2[b * NQ + j] * sa;
            }
        T[c] = sb;
    }
    for (int k = 0; k < NQ; ++k) {
        double s = 0.0;
        for (int a = 0; a < NQ; ++a) {
            s += sD2[a * NQ + i] * g(0, a + NQ * j, k);    // rr
            s += sD2[a * NQ + j] * g(3, i + NQ * a, k);    // ss
            s += sD2[a * NQ + k] * g(5, t, a);             // tt
        }
        s += 2.0 * sDd[i] * sDd[j] * g(1, t, k) + 2.0 * sDd[i] * sDd[k] * g(2, t, k) +
             2.0 * sDd[j] * sDd[k] * g(4, t, k);
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < NG; ++c) m += sI2[c * NQ + k] * T[c];
        dl[e * NP + t + NC * k] = s + lambda * m;
    }
}

template <int NQ>
static hipError_t elem_diag_launch(int64_t E, const double *D1d, const double *I1d, const double *G,
                                   const double *wJ, double lambda, double *dl, hipStream_t s)
{
    // one element per workgroup, split over launches of at most max_grid workgroups
    constexpr int threads = round_up_wave(NQ * NQ);
    for (int64_t e0 = 0; e0 < E; e0 += max_grid(threads)) {
        const int64_t grid = E - e0 < max_grid(threads) ? E - e0 : max_grid(threads);
        hipLaunchKernelGGL((elem_diag_kernel<NQ>), dim3(static_cast<unsigned>(grid)), dim3(threads), 0, s, E, D1d,
                           I1d, G, wJ, lambda, dl, e0);
    }
    return hipGetLastError();
}

hipError_t launch_elem_diag(int N, int64_t E, const double *D1d, const double *I1d, const double *G,
                            const double *wJ, double lambda, double *dl, hipStream_t s)
{
    if (E < 1) return hipSuccess;
    switch (N + 1) {
#define FEM_DIAG(q) case q: return elem_diag_launch<q>(E, D1d, I1d, G, wJ, lambda, dl, s);
        FEM_DIAG(2) FEM_DIAG(3) FEM_DIAG(4) FEM_DIAG(5) FEM_DIAG(6) FEM_DIAG(7) FEM_DIAG(8) FEM_DIAG(9)
        FEM_DIAG(10) FEM_DIAG(11) FEM_DIAG(12) FEM_DIAG(13) FEM_DIAG(14) FEM_DIAG(15) FEM_DIAG(16)
#undef FEM_DIAG
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather(const int32_t *gid, const double *ug, double *ul, int64_t nl, int64_t ng, hipStream_t s)
{
    if (nl < 1) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>(as_blocks(nl))), dim3(kAsThreads), 0, s, gid, ug,
                       ul, nl, ng);
    return hipGetLastError();
}

hipError_t launch_scatter(const int32_t *off, const int32_t *loc, const double *ul, double *ug, int64_t ng,
                          int64_t nl, const double *pdot, double *part, hipStream_t s)
{
    if (ng < 1) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3(static_cast<unsigned>(as_blocks(ng))), dim3(kAsThreads), 0, s, off,
                       loc, ul, ug, ng, nl, pdot, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jacobi-preconditioned CG on the global vectors (FP64).
// ---------------------------------------------------------------------------
struct PcgScalars {
    double rz;       // r . z of the current direction
    double rz_new;
    double pAp;
    double alpha;
    double beta;
    double rr;       // recursive ||r||^2 after the last update
    double true_rr;  // ||b - A x||^2 at the last true-residual check
    double bb;
};

// One workgroup sums n partials (fixed order) into *out, then a scalar step.
enum { PFIN_PLAIN = 0, PFIN_ALPHA = 1, PFIN_BETA = 2 };
__global__ __launch_bounds__(kAsThreads) void pcg_finalize_kernel(const double *__restrict__ part, int64_t n,
                                                                  double *out, PcgScalars *sc, int what)
{
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kAsThreads) s += part[i];
    s = wg_sum(s);
    if (threadIdx.x == 0) {
        *out = s;
        if (what == PFIN_ALPHA) sc->alpha = sc->rz / s;
        if (what == PFIN_BETA) {
            sc->beta = s / sc->rz;
            sc->rz = s;
        }
    }
}

// dinv = 1 / diag, or 1 without a preconditioner
__global__ __launch_bounds__(kAsThreads) void pcg_recip_kernel(const double *__restrict__ diag,
                                                               double *__restrict__ dinv, int64_t n)
{
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g < n) dinv[g] = diag ? 1.0 / diag[g] : 1.0;
    }
}

// r = b - Ax; partials of r.r, r.z (z = dinv r) and b.b; with p set, p = z.
__global__ __launch_bounds__(kAsThreads) void pcg_residual_kernel(
    const double *__restrict__ b, const double *__restrict__ Ax, const double *__restrict__ dinv,
    double *__restrict__ r, double *__restrict__ p, int64_t n, double *__restrict__ part_rr,
    double *__restrict__ part_rz, double *__restrict__ part_bb)
{
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
    double srr = 0.0, srz = 0.0, sbb = 0.0;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g >= n) continue;
        const double bv = b[g];
        const double v = bv - Ax[g];
        const double z = dinv[g] * v;
        r[g] = v;
        if (p) p[g] = z;
        srr += v * v;
        srz += v * z;
        sbb += bv * bv;
    }
    srr = wg_sum(srr);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = srr;
    srz = wg_sum(srz);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = srz;
    sbb = wg_sum(sbb);
    if (threadIdx.x == 0) part_bb[blockIdx.x] = sbb;
}

// x += alpha p; r -= alpha Ap; partials of r.z and r.r.
__global__ __launch_bounds__(kAsThreads) void pcg_update_kernel(
    double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p, const double *__restrict__ Ap,
    const double *__restrict__ dinv, int64_t n, const PcgScalars *__restrict__ sc, double *__restrict__ part_rz,
    double *__restrict__ part_rr)
{
    const double alpha = sc->alpha;
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
    double pv[kAsPer], av[kAsPer], xv[kAsPer], rv[kAsPer], dv[kAsPer];
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g < n) {
            pv[q] = p[g];
            av[q] = Ap[g];
            xv[q] = x[g];
            rv[q] = r[g];
            dv[q] = dinv[g];
        }
    }
    double srz = 0.0, srr = 0.0;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g < n) {
            xv[q] += alpha * pv[q];
            rv[q] -= alpha * av[q];
            x[g] = xv[q];
            r[g] = rv[q];
            srz += rv[q] * (dv[q] * rv[q]);
            srr += rv[q] * rv[q];
        }
    }
    srz = wg_sum(srz);
    if (threadIdx.x == 0) part_rz[blockIdx.x] = srz;
    srr = wg_sum(srr);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = srr;
}

// p = dinv r + beta p
__global__ __launch_bounds__(kAsThreads) void pcg_direction_kernel(double *__restrict__ p,
                                                                   const double *__restrict__ r,
                                                                   const double *__restrict__ dinv, int64_t n,
                                                                   const PcgScalars *__restrict__ sc)
{
    const double beta = sc->beta;
    const int64_t base = blockIdx.x * kAsChunk + threadIdx.x;
#pragma unroll
    for (int q = 0; q < kAsPer; ++q) {
        const int64_t g = base + q * kAsThreads;
        if (g < n) p[g] = dinv[g] * r[g] + beta * p[g];
    }
}

namespace {

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

struct AsLayout {
    size_t pl, yl, r, p, Ap, dinv, part, sc, total;
};

AsLayout as_layout(int64_t nl, int64_t ng)
{
    AsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.pl = take(static_cast<size_t>(nl) * 8);
    L.yl = take(static_cast<size_t>(nl) * 8);
    L.r = take(static_cast<size_t>(ng) * 8);
    L.p = take(static_cast<size_t>(ng) * 8);
    L.Ap = take(static_cast<size_t>(ng) * 8);
    L.dinv = take(static_cast<size_t>(ng) * 8);
    L.part = take(static_cast<size_t>(3 * as_blocks(ng)) * 8);
    L.sc = take(sizeof(PcgScalars));
    L.total = off;
    return L;
}

// yl = (S + lambda M) pl with the element kernels (FP64, tuned packings)
hipError_t apply_local(const fem_cg_operator *op, const double *pl, double *yl, hipStream_t s)
{
    ApplyArgs a{};
    a.N = op->N;
    a.E = op->E;
    a.I1d = op->I1d;
    a.D1d = op->D1d;
    a.u = pl;
    a.y = yl;
    a.prec = P_F64;
    a.op = OP_BP35;
    a.G = op->G;
    a.geo_scale = 1.0f;
    fem_tune_get(OP_BP35, a.N, P_F64, &a.epb, &a.grid_cap);
    hipError_t e = launch_bp35(a, s);
    if (e != hipSuccess || op->lambda == 0.0) return e;
    a.op = OP_BP10;
    a.G = nullptr;
    a.wJ = op->wJ;
    a.beta = 1.0;
    a.out_scale = op->lambda;
    fem_tune_get(OP_BP10, a.N, P_F64, &a.epb, &a.grid_cap);
    return launch_bp10(a, s);
}

}  // namespace

size_t assembled_workspace_bytes(const fem_cg_operator *op, const fem_assembly *as)
{
    const int64_t nl = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    return as_layout(nl, as->n_global).total;
}

// yg = Z^T (S + lambda M) Z ug; with pdot set, partials of pdot . yg into part.
static hipError_t assembled_apply_ws(const fem_cg_operator *op, const fem_assembly *as, const double *ug,
                                     double *yg, char *ws, const double *pdot, double *part, hipStream_t s)
{
    const int64_t nl = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    const AsLayout L = as_layout(nl, as->n_global);
    double *pl = reinterpret_cast<double *>(ws + L.pl);
    double *yl = reinterpret_cast<double *>(ws + L.yl);
    hipError_t e = launch_gather(as->gather, ug, pl, nl, as->n_global, s);
    if (e == hipSuccess) e = apply_local(op, pl, yl, s);
    if (e == hipSuccess) e = launch_scatter(as->offsets, as->locals, yl, yg, as->n_global, nl, pdot, part, s);
    return e;
}

int assembled_apply(const fem_cg_operator *op, const fem_assembly *as, const double *ug, double *yg, void *ws,
                    hipStream_t s)
{
    return assembled_apply_ws(op, as, ug, yg, static_cast<char *>(ws), nullptr, nullptr, s) == hipSuccess
               ? FEM_OK
               : FEM_ERR_HIP;
}

int assembled_diagonal(const fem_cg_operator *op, const fem_assembly *as, double *diag, void *ws, hipStream_t s)
{
    const int64_t nl = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    const AsLayout L = as_layout(nl, as->n_global);
    double *yl = reinterpret_cast<double *>(static_cast<char *>(ws) + L.yl);
    hipError_t e = launch_elem_diag(op->N, op->E, op->D1d, op->I1d, static_cast<const double *>(op->G),
                                    static_cast<const double *>(op->wJ), op->lambda, yl, s);
    if (e == hipSuccess)
        e = launch_scatter(as->offsets, as->locals, yl, diag, as->n_global, nl, nullptr, nullptr, s);
    return e == hipSuccess ? FEM_OK : FEM_ERR_HIP;
}

int pcg_solve(const fem_cg_operator *op, const fem_assembly *as, const fem_cg_options *opt, const double *diag,
              const double *b, double *x, void *ws, fem_cg_report *rep, hipStream_t s)
{
    const int64_t nl = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    const int64_t ng = as->n_global;
    const AsLayout L = as_layout(nl, ng);
    char *w = static_cast<char *>(ws);
    double *r = reinterpret_cast<double *>(w + L.r);
    double *p = reinterpret_cast<double *>(w + L.p);
    double *Ap = reinterpret_cast<double *>(w + L.Ap);
    double *dinv = reinterpret_cast<double *>(w + L.dinv);
    const int64_t nb = as_blocks(ng);
    double *part1 = reinterpret_cast<double *>(w + L.part);
    double *part2 = part1 + nb;
    double *part3 = part2 + nb;
    PcgScalars *sc = reinterpret_cast<PcgScalars *>(w + L.sc);
    const dim3 grid(static_cast<unsigned>(nb)), block(kAsThreads);
    const auto t0 = std::chrono::steady_clock::now();
    PcgScalars h{};
    auto fetch = [&]() -> bool {
        return hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    auto fin = [&](const double *pp, double *out, int what) {
        hipLaunchKernelGGL(pcg_finalize_kernel, dim3(1), block, 0, s, pp, nb, out, sc, what);
    };
    auto record = [&](double rel) {
        if (opt->history && rep->history_count < opt->history_len) opt->history[rep->history_count++] = rel;
    };
    // true residual r = b - A x and the direction p = z restarted from it
    auto restart = [&]() -> bool {
        if (assembled_apply_ws(op, as, x, Ap, w, nullptr, nullptr, s) != hipSuccess) return false;
        hipLaunchKernelGGL(pcg_residual_kernel, grid, block, 0, s, b, Ap, dinv, r, p, ng, part1, part2, part3);
        fin(part1, &sc->true_rr, PFIN_PLAIN);
        fin(part2, &sc->rz, PFIN_PLAIN);
        fin(part3, &sc->bb, PFIN_PLAIN);
        rep->hi_matvecs += 1;
        return hipGetLastError() == hipSuccess && fetch();
    };

    rep->iters = 0;
    rep->reliable_updates = 0;
    rep->hi_matvecs = 0;
    rep->history_count = 0;
    rep->status = FEM_OK;
    if (hipMemsetAsync(sc, 0, sizeof(PcgScalars), s) != hipSuccess) return FEM_ERR_HIP;
    hipLaunchKernelGGL(pcg_recip_kernel, grid, block, 0, s, diag, dinv, ng);
    if (!restart()) return FEM_ERR_HIP;
    const double bnorm = std::sqrt(h.bb);
    const double target = opt->rtol * bnorm;
    double rel = bnorm > 0 ? std::sqrt(h.true_rr) / bnorm : 0.0;
    record(rel);
    bool converged = std::sqrt(h.true_rr) <= target || bnorm == 0.0;
    const int every = opt->check_every > 0 ? opt->check_every : 1;
    // A recursive residual at or below check_at triggers a true-residual
    // check.  When the check fails (the true residual sits at its rounding
    // floor), the solve restarts from the true residual and the next check
    // waits until the recursion has halved the residual of the failed check.
    double check_at = target;
    bool fresh = true;   // p was just set to z: no direction update
    int it = 0;
    while (!converged && it < opt->max_iters) {
        ++it;
        if (!fresh) hipLaunchKernelGGL(pcg_direction_kernel, grid, block, 0, s, p, r, dinv, ng, sc);
        fresh = false;
        if (assembled_apply_ws(op, as, p, Ap, w, p, part1, s) != hipSuccess) return FEM_ERR_HIP;
        fin(part1, &sc->pAp, PFIN_ALPHA);
        hipLaunchKernelGGL(pcg_update_kernel, grid, block, 0, s, x, r, p, Ap, dinv, ng, sc, part2, part3);
        fin(part3, &sc->rr, PFIN_PLAIN);
        fin(part2, &sc->rz_new, PFIN_BETA);
        if (hipGetLastError() != hipSuccess) return FEM_ERR_HIP;
        if (it % every == 0 || it == opt->max_iters) {
            if (!fetch()) return FEM_ERR_HIP;
            if (!(h.pAp > 0.0) || !std::isfinite(h.rr)) {
                rep->status = FEM_ERR_BREAKDOWN;
                break;
            }
            const double rn = std::sqrt(h.rr);
            if (rn <= check_at) {
                if (!restart()) return FEM_ERR_HIP;
                rep->reliable_updates += 1;
                rel = std::sqrt(h.true_rr) / bnorm;
                record(rel);
                if (std::sqrt(h.true_rr) <= target) {
                    converged = true;
                    break;
                }
                fresh = true;
                check_at = 0.5 * rn;
            }
        }
    }
    if (!converged) {
        if (!restart()) return FEM_ERR_HIP;
        rel = std::sqrt(h.true_rr) / bnorm;
        record(rel);
        converged = std::sqrt(h.true_rr) <= target;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return FEM_ERR_HIP;
    const auto t1 = std::chrono::steady_clock::now();
    rep->iters = it > opt->max_iters ? opt->max_iters : it;
    rep->rel_res = rel;
    rep->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (rep->status == FEM_OK && !converged) rep->status = FEM_ERR_NOT_CONVERGED;
    return rep->status;
}

}  // namespace fem
