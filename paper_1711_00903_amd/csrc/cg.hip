// cg.hip -- conjugate gradients on the unassembled screened-Poisson operator
// A = S(BP3.5) + lambda M(BP1.0) (Problem description section: the global
// operator is block diagonal and symmetric positive definite for lambda > 0).
//
// One code path serves every arm:
//   * FP64 CG: iterates, operator and vectors in FP64;
//   * mixed precision (mode 1): the Krylov iteration runs with an operator
//     whose geometric data is stored in FP32, BF16 or FP16, and either FP64
//     vectors and arithmetic (the *G64 storage modes) or FP32 vectors and
//     arithmetic (FEM_F32, FEM_BF16G, FEM_F16G);
//   * iterative refinement (mode 2): as mode 1, with the Krylov iteration
//     restarted at every reliable update (an inner CG per refinement step);
// and all use reliable updates (residual replacement, Sleijpen & van der
// Vorst 1996; the mixed-precision form of Clark et al. 2010): the iterate is
// accumulated in the iteration precision since the last update, and whenever
// the recursive residual has dropped by `delta` relative to the last true
// residual, x += x_lo and r = b - A x are recomputed in FP64.  The solve stops
// on the FP64 true residual: ||b - A x|| <= rtol ||b||.
//
// Dot products accumulate in FP64 with a fixed two-stage reduction (per-block
// partials, then one block), so a solve is bitwise repeatable.
#include <chrono>
#include <cmath>
#include <cstring>

#include "cgop.hpp"
#include "fem.h"
#include "fem_device.hpp"
#include "launch.hpp"

namespace fem {

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

struct CgScalars {
    double rr;       // r_lo . r_lo of the current iterate
    double rr_new;   // after the update
    double pAp;
    double alpha;
    double beta;
    double true_rr;  // ||b - A x||^2 at the last reliable update
    double bb;       // ||b||^2
    double pad;
};

__device__ __forceinline__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

template <class TA, class TB>
__global__ __launch_bounds__(kRedThreads) void dot_kernel(const TA *__restrict__ a, const TB *__restrict__ b,
                                                          int64_t n, double *__restrict__ part)
{
    __shared__ double sh[kRedThreads];
    double s = 0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads)
        s += static_cast<double>(a[i]) * static_cast<double>(b[i]);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Partial sums of v[0..n) per block, in a fixed order.
__global__ __launch_bounds__(kRedThreads) void sum_kernel(const double *__restrict__ v, int64_t n,
                                                          double *__restrict__ part)
{
    __shared__ double sh[kRedThreads];
    double s = 0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads)
        s += v[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Final reduction of kRedBlocks partials into *out, then a scalar step:
//   what == 0: out = rr (nothing else)
//   what == 1: pAp: alpha = rr / pAp
//   what == 2: rr_new: beta = rr_new / rr, rr = rr_new
enum { FIN_PLAIN = 0, FIN_ALPHA = 1, FIN_BETA = 2 };
__global__ __launch_bounds__(kRedThreads) void finalize_kernel(const double *__restrict__ part, int64_t n,
                                                               double *out, CgScalars *sc, int what)
{
    __shared__ double sh[kRedThreads];
    double s = 0;
    for (int64_t i = threadIdx.x; i < n; i += kRedThreads) s += part[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) {
        *out = s;
        if (what == FIN_ALPHA) sc->alpha = sc->rr / s;
        if (what == FIN_BETA) {
            sc->beta = s / sc->rr;
            sc->rr = s;
        }
    }
}

// x_lo += alpha p (unless UPD_X is false: the two-kernel step folds it into
// the next direction update); r_lo -= alpha Ap; per-block partial sums of
// r_lo . r_lo.
// Non-persistent: block b owns kUpdPairs * kRedThreads consecutive pairs of
// entries (16-byte vectors for FP64), every thread issues all its loads before
// its first store (the streaming-copy pattern; a grid-stride loop over the
// same data reaches only 4.7 TB/s).  The odd last entry goes to the last
// block's thread 0.
constexpr int kUpdPairs = 4;
constexpr int64_t kUpdBlockPairs = static_cast<int64_t>(kUpdPairs) * kRedThreads;

inline int64_t update_blocks(int64_t n)
{
    const int64_t b = (n / 2 + kUpdBlockPairs - 1) / kUpdBlockPairs;
    return b > 0 ? b : 1;
}

template <class TV, bool UPD_X = true>
__global__ __launch_bounds__(kRedThreads) void update_kernel(TV *__restrict__ xl, TV *__restrict__ rl,
                                                             const TV *__restrict__ p,
                                                             const TV *__restrict__ Ap, int64_t n,
                                                             const CgScalars *__restrict__ sc,
                                                             double *__restrict__ part)
{
    __shared__ double sh[kRedThreads];
    const TV alpha = static_cast<TV>(sc->alpha);
    using V2 = TV __attribute__((ext_vector_type(2)));
    const int64_t n2 = n / 2;
    V2 *x2 = reinterpret_cast<V2 *>(xl);
    V2 *r2 = reinterpret_cast<V2 *>(rl);
    const V2 *p2 = reinterpret_cast<const V2 *>(p);
    const V2 *a2 = reinterpret_cast<const V2 *>(Ap);
    const int64_t i0 = blockIdx.x * kUpdBlockPairs + threadIdx.x;
    V2 pv[kUpdPairs], av[kUpdPairs], xv[kUpdPairs], rv[kUpdPairs];
#pragma unroll
    for (int q = 0; q < kUpdPairs; ++q) {
        const int64_t i = i0 + q * kRedThreads;
        if (i < n2) {
            if constexpr (UPD_X) {
                pv[q] = p2[i];
                xv[q] = x2[i];
            }
            av[q] = a2[i];
            rv[q] = r2[i];
        }
    }
    double s = 0;
#pragma unroll
    for (int q = 0; q < kUpdPairs; ++q) {
        const int64_t i = i0 + q * kRedThreads;
        if (i < n2) {
            rv[q] -= alpha * av[q];
            if constexpr (UPD_X) {
                xv[q] += alpha * pv[q];
                x2[i] = xv[q];
            }
            r2[i] = rv[q];
            s += static_cast<double>(rv[q].x) * static_cast<double>(rv[q].x);
            s += static_cast<double>(rv[q].y) * static_cast<double>(rv[q].y);
        }
    }
    if ((n & 1) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const int64_t i = n - 1;
        if constexpr (UPD_X) xl[i] += alpha * p[i];
        const TV r = rl[i] - alpha * Ap[i];
        rl[i] = r;
        s += static_cast<double>(r) * static_cast<double>(r);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = r_lo + beta p
template <class TV>
__global__ __launch_bounds__(kRedThreads) void xpay_kernel(TV *__restrict__ p, const TV *__restrict__ rl,
                                                           int64_t n, const CgScalars *__restrict__ sc)
{
    const TV beta = static_cast<TV>(sc->beta);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads)
        p[i] = rl[i] + beta * p[i];
}

// x_lo += alpha p: the iterate update still pending from a two-kernel step
template <class TV>
__global__ __launch_bounds__(kRedThreads) void axpy_kernel(TV *__restrict__ xl, const TV *__restrict__ p,
                                                           int64_t n, const CgScalars *__restrict__ sc)
{
    const TV alpha = static_cast<TV>(sc->alpha);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads)
        xl[i] += alpha * p[i];
}

// x += x_lo; x_lo = 0
template <class TV>
__global__ __launch_bounds__(kRedThreads) void merge_kernel(double *__restrict__ x, TV *__restrict__ xl, int64_t n)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads) {
        x[i] += static_cast<double>(xl[i]);
        xl[i] = TV(0);
    }
}

// r = b - Ax (FP64); r_lo = (TV) r; optionally p = r_lo; partials of r.r and r_lo.r_lo
template <class TV>
__global__ __launch_bounds__(kRedThreads) void residual_kernel(const double *__restrict__ b,
                                                               const double *__restrict__ Ax,
                                                               double *__restrict__ r, TV *__restrict__ rl,
                                                               TV *__restrict__ p, int64_t n,
                                                               double *__restrict__ part_true,
                                                               double *__restrict__ part_lo)
{
    __shared__ double sh[kRedThreads];
    double st = 0, sl = 0;
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads) {
        const double v = b[i] - Ax[i];
        r[i] = v;
        const TV w = static_cast<TV>(v);
        rl[i] = w;
        if (p) p[i] = w;
        st += v * v;
        sl += static_cast<double>(w) * static_cast<double>(w);
    }
    st = block_sum(st, sh);
    if (threadIdx.x == 0) part_true[blockIdx.x] = st;
    __syncthreads();
    sl = block_sum(sl, sh);
    if (threadIdx.x == 0) part_lo[blockIdx.x] = sl;
}

template <class TV>
__global__ __launch_bounds__(kRedThreads) void fill_kernel(TV *__restrict__ v, int64_t n)
{
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kRedThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kRedThreads)
        v[i] = TV(0);
}

// ---------------------------------------------------------------------------
// Host driver.
// ---------------------------------------------------------------------------
hipError_t launch_cgop_f64(const CgopArgs &, hipStream_t);
hipError_t launch_cgop_f32g64(const CgopArgs &, hipStream_t);
hipError_t launch_cgop_bf16g64(const CgopArgs &, hipStream_t);
hipError_t launch_cgop_f16g64(const CgopArgs &, hipStream_t);

namespace {

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// Entries of the per-group partial-sum buffer: one per workgroup of the
// one-pass operator, one per element of the two-kernel form.
int64_t cg_groups(int N, int64_t E)
{
    const int64_t n = E * static_cast<int64_t>(N + 1) * (N + 1) * (N + 1);
    int64_t g = cgop_groups(N, E);
    if (E > g) g = E;
    if (update_blocks(n) > g) g = update_blocks(n);
    return g;
}

struct Layout {
    size_t r, tmp, xl, rl, p, Ap, part, partg, sc, total;
};

Layout layout(int64_t n, size_t vbytes, int64_t groups)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    L.r = take(n * 8);
    L.tmp = take(n * 8);
    L.xl = take(n * vbytes);
    L.rl = take(n * vbytes);
    L.p = take(n * vbytes);
    L.Ap = take(n * vbytes);
    L.part = take(3 * kRedBlocks * sizeof(double));
    L.partg = take(static_cast<size_t>(groups) * sizeof(double));
    L.sc = take(sizeof(CgScalars));
    L.total = off;
    return L;
}

bool check(hipError_t e) { return e == hipSuccess; }

struct Ctx {
    const fem_cg_operator *op;
    hipStream_t s;
    int64_t n;
    unsigned grid;
};

// y = A u with operator data in precision `prec` (FP64 vectors for FEM_F64,
// FP32 otherwise).
hipError_t apply_A(const Ctx &c, int prec, const void *u, void *y)
{
    const fem_cg_operator *op = c.op;
    const bool hi = prec == FEM_F64;   // the FP64 operator of the true residuals
    ApplyArgs a{};
    a.N = op->N;
    a.E = op->E;
    a.I1d = op->I1d;
    a.D1d = op->D1d;
    a.u = u;
    a.y = y;
    a.prec = prec;
    // stiffness: y = S u
    a.op = OP_BP35;
    a.G = hi ? op->G : op->G_lo;
    a.wJ = nullptr;
    a.lambda = 0.0;
    a.beta = 0.0;
    a.geo_scale = op->geo_scale_G;
    fem_tune_get(OP_BP35, a.N, prec, &a.epb, &a.grid_cap);
    hipError_t e = launch_bp35(a, c.s);
    if (e != hipSuccess || op->lambda == 0.0) return e;
    // mass: y += lambda M u
    a.op = OP_BP10;
    a.G = nullptr;
    a.wJ = hi ? op->wJ : op->wJ_lo;
    a.beta = 1.0;
    a.out_scale = op->lambda;
    a.geo_scale = op->geo_scale_wJ;
    fem_tune_get(OP_BP10, a.N, prec, &a.epb, &a.grid_cap);
    return launch_bp10(a, c.s);
}

// Two-kernel Krylov operator on FP64 or FP32 vectors: the stiffness kernel
// applies the direction update u <- r + (*beta) u as it loads u (when r is
// set), the mass kernel (one-wave BP1.0) adds lambda M u and writes
// per-element partials of u . y into epart.  Requires N <= 7 and lambda != 0.
hipError_t apply_A_split(const Ctx &c, int prec, const void *r, const double *beta, void *u, void *y,
                         double *epart, void *xl, const double *alpha)
{
    const fem_cg_operator *op = c.op;
    const bool hi = prec == FEM_F64;
    ApplyArgs a{};
    a.N = op->N;
    a.E = op->E;
    a.I1d = op->I1d;
    a.D1d = op->D1d;
    a.u = u;
    a.y = y;
    a.prec = prec;
    a.op = OP_BP35;
    a.G = hi ? op->G : op->G_lo;
    a.geo_scale = op->geo_scale_G;
    a.xr = r;
    a.xbeta = beta;
    a.xl = r ? xl : nullptr;
    a.xalpha = alpha;
    // the tuned packing, but the grid uncapped: a persistent grid chosen for
    // the plain apply does not carry over to this form, which also reads r and
    // x and writes u and x (BF16 factors, FP64 vectors, N = 7: 1.70 ms with
    // the plain apply's 1024 workgroups against 1.52 ms uncapped)
    int cap = 0;
    fem_tune_get(OP_BP35, a.N, prec, &a.epb, &cap);
    a.grid_cap = 0;
    hipError_t e = launch_bp35(a, c.s);
    if (e != hipSuccess) return e;
    a.op = OP_BP10;
    a.G = nullptr;
    a.wJ = hi ? op->wJ : op->wJ_lo;
    a.beta = 1.0;
    a.out_scale = op->lambda;
    a.geo_scale = op->geo_scale_wJ;
    a.xr = nullptr;
    a.xbeta = nullptr;
    a.xl = nullptr;
    a.xalpha = nullptr;
    a.part = epart;
    a.epb = 1;          // the one-wave kernel
    a.grid_cap = 0;
    return launch_bp10(a, c.s);
}

inline bool split_supported(int N) { return N + 1 <= 8; }

// One-pass operator y = A u (optionally u <- r + beta u first), FP64 fields,
// geometric data of precision `prec`; partials of u . y into part.
hipError_t apply_cgop(const Ctx &c, int prec, const double *r, double *u, const double *beta, int xpay,
                      double *y, double *part)
{
    const fem_cg_operator *op = c.op;
    const bool hi = prec == FEM_F64;
    CgopArgs a{};
    a.N = op->N;
    a.E = op->E;
    a.I1d = op->I1d;
    a.D1d = op->D1d;
    a.G = hi ? op->G : op->G_lo;
    a.wJ = hi ? op->wJ : op->wJ_lo;
    const bool f16 = is_f16_prec(prec);
    a.s_scale = f16 ? 1.0 / op->geo_scale_G : 1.0;
    a.m_scale = f16 ? op->lambda / op->geo_scale_wJ : op->lambda;
    a.r = r;
    a.p = u;
    a.beta = beta;
    a.do_xpay = xpay;
    a.Ap = y;
    a.part = part;
    switch (prec) {
    case FEM_F64: return launch_cgop_f64(a, c.s);
    case FEM_F32G64: return launch_cgop_f32g64(a, c.s);
    case FEM_BF16G64: return launch_cgop_bf16g64(a, c.s);
    case FEM_F16G64: return launch_cgop_f16g64(a, c.s);
    default: return hipErrorInvalidValue;
    }
}

template <class TV>
int solve_t(const fem_cg_operator *op, const fem_cg_options *opt, int prec_lo, const double *b, double *x,
            void *ws, fem_cg_report *rep, hipStream_t s)
{
    const int64_t np = static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    const int64_t n = op->E * np;
    const int64_t groups = cg_groups(op->N, op->E);
    const Layout L = layout(n, sizeof(TV), groups);
    // the one-pass form needs FP64 vectors and a mass term, the two-kernel
    // form a mass term
    const bool f64v = std::is_same<TV, double>::value && op->lambda != 0.0;
    const bool fused = f64v && opt->fusion == FEM_CG_FUSE_ONEPASS && cgop_supported(op->N);
    const bool split = op->lambda != 0.0 && opt->fusion == FEM_CG_FUSE_AUTO && split_supported(op->N);
    char *w = static_cast<char *>(ws);
    double *r = reinterpret_cast<double *>(w + L.r);
    double *tmp = reinterpret_cast<double *>(w + L.tmp);
    TV *xl = reinterpret_cast<TV *>(w + L.xl);
    TV *rl = reinterpret_cast<TV *>(w + L.rl);
    TV *p = reinterpret_cast<TV *>(w + L.p);
    TV *Ap = reinterpret_cast<TV *>(w + L.Ap);
    double *part = reinterpret_cast<double *>(w + L.part);
    double *part2 = part + kRedBlocks;
    double *part3 = part + 2 * kRedBlocks;
    double *partg = reinterpret_cast<double *>(w + L.partg);
    CgScalars *sc = reinterpret_cast<CgScalars *>(w + L.sc);
    Ctx c{op, s, n, kRedBlocks};
    const dim3 G(kRedBlocks), B(kRedThreads);
    const auto t0 = std::chrono::steady_clock::now();
    CgScalars h{};
    auto fetch = [&]() -> bool {
        if (!check(hipMemcpyAsync(&h, sc, sizeof(h), hipMemcpyDeviceToHost, s))) return false;
        return check(hipStreamSynchronize(s));
    };
    auto fin = [&](const double *pp, int64_t cnt, double *out, int what) {
        hipLaunchKernelGGL(finalize_kernel, dim3(1), B, 0, s, pp, cnt, out, sc, what);
    };
    // FP64 operator applied to x into tmp
    auto apply_hi = [&]() -> hipError_t {
        if (fused) return apply_cgop(c, FEM_F64, nullptr, x, nullptr, 0, tmp, partg);
        return apply_A(c, FEM_F64, x, tmp);
    };
    // true residual r = b - A x; r_lo = (TV) r.  At the start (set_p) also
    // p = r_lo and rr = r_lo.r_lo; at a reliable update the replaced r_lo.r_lo
    // goes to rr_new and its partials stay in part2, where the beta step below
    // reads them (beta = replaced rr / previous rr).
    auto true_residual = [&](bool set_p) -> hipError_t {
        hipError_t e = apply_hi();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(residual_kernel<TV>, G, B, 0, s, b, tmp, r, rl, set_p ? p : nullptr, n, part,
                           part2);
        fin(part, kRedBlocks, &sc->true_rr, FIN_PLAIN);
        fin(part2, kRedBlocks, set_p ? &sc->rr : &sc->rr_new, FIN_PLAIN);
        return hipGetLastError();
    };
    auto record = [&](double rel) {
        if (opt->history && rep->history_count < opt->history_len) opt->history[rep->history_count++] = rel;
    };

    rep->iters = 0;
    rep->reliable_updates = 0;
    rep->hi_matvecs = 0;
    rep->history_count = 0;
    rep->status = FEM_OK;
    if (!check(hipMemsetAsync(sc, 0, sizeof(CgScalars), s))) return FEM_ERR_HIP;
    hipLaunchKernelGGL((dot_kernel<double, double>), G, B, 0, s, b, b, n, part3);
    fin(part3, kRedBlocks, &sc->bb, FIN_PLAIN);
    hipLaunchKernelGGL(fill_kernel<TV>, G, B, 0, s, xl, n);
    if (true_residual(true) != hipSuccess) return FEM_ERR_HIP;
    rep->hi_matvecs = 1;
    if (!fetch()) return FEM_ERR_HIP;
    const double bnorm = std::sqrt(h.bb);
    const double target = opt->rtol * bnorm;
    double rmax = std::sqrt(h.true_rr);
    double rel = bnorm > 0 ? rmax / bnorm : 0.0;
    record(rel);
    const double delta = opt->delta > 0 ? opt->delta : 0.1;
    const int every = opt->check_every > 0 ? opt->check_every : 1;
    bool converged = rmax <= target || bnorm == 0.0;
    // A recursive residual below the target triggers a true-residual check;
    // when that check fails (the true residual sits at its rounding floor while
    // the recursion keeps falling), the next such check waits until the
    // recursive residual has halved again, so checks do not repeat every step.
    double check_at = target;
    // mode 2 (iterative refinement): every reliable update also restarts the
    // Krylov iteration from the replaced residual (p = r_lo, no direction
    // update in the next step), so each refinement step is a fresh inner CG
    // in the low precision, stopped when it has reduced the residual by delta
    const bool restart_ir = opt->mode == 2;
    bool fresh = true;   // p = r_lo already: no direction update in the next step
    // two-kernel step: the update kernel leaves x_lo alone and the next
    // direction update adds alpha p into it; `pending` marks a step whose
    // alpha p is still to be added (flushed before x_lo is used or p replaced)
    bool pending = false;
    auto flush = [&]() {
        if (pending) hipLaunchKernelGGL(axpy_kernel<TV>, G, B, 0, s, xl, p, n, sc);
        pending = false;
    };
    int it = 0;
    while (!converged && it < opt->max_iters) {
        ++it;
        const bool xpay = !fresh;
        fresh = false;
        if (fused) {
            // p <- r_lo + beta p (except right after a (re)start), Ap, p . Ap
            if (apply_cgop(c, prec_lo, reinterpret_cast<const double *>(rl), reinterpret_cast<double *>(p),
                           &sc->beta, xpay, reinterpret_cast<double *>(Ap), partg) != hipSuccess)
                return FEM_ERR_HIP;
            fin(partg, cgop_groups(op->N, op->E), &sc->pAp, FIN_ALPHA);
        } else if (split) {
            if (!xpay) flush();
            if (apply_A_split(c, prec_lo, xpay ? rl : nullptr, &sc->beta, p, Ap, partg, pending ? xl : nullptr,
                              &sc->alpha) != hipSuccess)
                return FEM_ERR_HIP;
            pending = false;
            hipLaunchKernelGGL(sum_kernel, G, B, 0, s, partg, op->E, part);
            fin(part, kRedBlocks, &sc->pAp, FIN_ALPHA);
        } else {
            if (xpay) hipLaunchKernelGGL(xpay_kernel<TV>, G, B, 0, s, p, rl, n, sc);
            if (apply_A(c, prec_lo, p, Ap) != hipSuccess) return FEM_ERR_HIP;
            hipLaunchKernelGGL((dot_kernel<TV, TV>), G, B, 0, s, p, Ap, n, part);
            fin(part, kRedBlocks, &sc->pAp, FIN_ALPHA);
        }
        if (split) {
            hipLaunchKernelGGL((update_kernel<TV, false>), dim3(static_cast<unsigned>(update_blocks(n))), B, 0, s,
                               xl, rl, p, Ap, n, sc, partg);
            pending = true;
        } else {
            hipLaunchKernelGGL((update_kernel<TV, true>), dim3(static_cast<unsigned>(update_blocks(n))), B, 0, s,
                               xl, rl, p, Ap, n, sc, partg);
        }
        hipLaunchKernelGGL(sum_kernel, G, B, 0, s, partg, update_blocks(n), part2);
        fin(part2, kRedBlocks, &sc->rr_new, FIN_PLAIN);
        if (it % every == 0 || it == opt->max_iters) {
            if (!fetch()) return FEM_ERR_HIP;
            if (!(h.pAp > 0.0) || !std::isfinite(h.rr_new)) {
                rep->status = FEM_ERR_BREAKDOWN;
                break;
            }
            const double rn = std::sqrt(h.rr_new);
            if (rn < delta * rmax || rn <= check_at) {
                const bool by_target = !(rn < delta * rmax);
                // reliable update: fold the low-precision iterate into x and
                // replace the recursive residual by the true one
                flush();
                hipLaunchKernelGGL(merge_kernel<TV>, G, B, 0, s, x, xl, n);
                if (true_residual(restart_ir) != hipSuccess) return FEM_ERR_HIP;
                fresh = restart_ir;
                rep->reliable_updates += 1;
                rep->hi_matvecs += 1;
                if (!fetch()) return FEM_ERR_HIP;
                rmax = std::sqrt(h.true_rr);
                rel = rmax / bnorm;
                record(rel);
                if (rmax <= target) {
                    converged = true;
                    break;
                }
                check_at = by_target ? 0.5 * rn : target;
            }
        }
        // beta = rr_new / rr; rr = rr_new (the direction update itself is
        // applied at the start of the next iteration; after a restart p and rr
        // are already set)
        if (!fresh) fin(part2, kRedBlocks, &sc->rr_new, FIN_BETA);
        if (hipGetLastError() != hipSuccess) return FEM_ERR_HIP;
    }
    if (!converged) {
        // fold in the last low-precision iterate and report the true residual
        flush();
        hipLaunchKernelGGL(merge_kernel<TV>, G, B, 0, s, x, xl, n);
        if (true_residual(false) != hipSuccess) return FEM_ERR_HIP;
        rep->hi_matvecs += 1;
        if (!fetch()) return FEM_ERR_HIP;
        rel = std::sqrt(h.true_rr) / bnorm;
        record(rel);
        converged = std::sqrt(h.true_rr) <= target;
    }
    if (!check(hipStreamSynchronize(s))) return FEM_ERR_HIP;
    const auto t1 = std::chrono::steady_clock::now();
    rep->iters = it;
    rep->rel_res = rel;
    rep->ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (rep->status == FEM_OK && !converged) rep->status = FEM_ERR_NOT_CONVERGED;
    return rep->status;
}

}  // namespace

size_t cg_workspace_bytes(const fem_cg_operator *op, const fem_cg_options *opt)
{
    const int64_t np = static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    return layout(op->E * np, (opt->mode == 0 || f64_fields(op->inner_prec)) ? 8 : 4,
                  cg_groups(op->N, op->E)).total;
}

int cg_solve(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x, void *ws,
             fem_cg_report *rep, hipStream_t s)
{
    // modes 1 and 2 differ only in the restart at a reliable update
    if (opt->mode == 0) return solve_t<double>(op, opt, FEM_F64, b, x, ws, rep, s);
    if (f64_fields(op->inner_prec)) return solve_t<double>(op, opt, op->inner_prec, b, x, ws, rep, s);
    return solve_t<float>(op, opt, op->inner_prec, b, x, ws, rep, s);
}

}  // namespace fem
