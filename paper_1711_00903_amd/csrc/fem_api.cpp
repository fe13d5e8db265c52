// fem_api.cpp -- the extern "C" entry points of libfem (declared in fem.h):
// argument validation (before anything is enqueued), dispatch to the kernel
// families by (operator, degree, storage precision), and the process-wide
// launch-configuration table.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fem.h"
#include "launch.hpp"
#include "tiles.hpp"

namespace fem {

hipError_t launch_bp35v(int N, int64_t E, const double *D1d, const double *X, double lambda, const double *u,
                        double *y, double beta, int64_t grid_cap, hipStream_t s);
hipError_t launch_bp30v(int N, int64_t E, const double *I1d, const double *Dgl, const double *X, double lambda,
                        const double *u, double *y, double beta, hipStream_t s);
hipError_t launch_bp35_f64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_f32(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_bf16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_f16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_bf16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_f16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_f32g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_bf16g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp35_f16g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f32(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_bf16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_bf16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f32g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_bf16g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp10_f16g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f32(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_bf16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f16(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_bf16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f16g(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f32g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_bf16g64(const ApplyArgs &, hipStream_t);
hipError_t launch_bp30_f16g64(const ApplyArgs &, hipStream_t);

hipError_t launch_bp35(const ApplyArgs &a, hipStream_t s)
{
    switch (a.prec) {
    case P_F64: return launch_bp35_f64(a, s);
    case P_F32: return launch_bp35_f32(a, s);
    case P_BF16: return launch_bp35_bf16(a, s);
    case P_F16: return launch_bp35_f16(a, s);
    case P_BF16G: return launch_bp35_bf16g(a, s);
    case P_F16G: return launch_bp35_f16g(a, s);
    case P_F32G64: return launch_bp35_f32g64(a, s);
    case P_BF16G64: return launch_bp35_bf16g64(a, s);
    case P_F16G64: return launch_bp35_f16g64(a, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_bp10(const ApplyArgs &a, hipStream_t s)
{
    switch (a.prec) {
    case P_F64: return launch_bp10_f64(a, s);
    case P_F32: return launch_bp10_f32(a, s);
    case P_BF16: return launch_bp10_bf16(a, s);
    case P_F16: return launch_bp10_f16(a, s);
    case P_BF16G: return launch_bp10_bf16g(a, s);
    case P_F16G: return launch_bp10_f16g(a, s);
    case P_F32G64: return launch_bp10_f32g64(a, s);
    case P_BF16G64: return launch_bp10_bf16g64(a, s);
    case P_F16G64: return launch_bp10_f16g64(a, s);
    default: return hipErrorInvalidValue;
    }
}
hipError_t launch_bp30(const ApplyArgs &a, hipStream_t s)
{
    switch (a.prec) {
    case P_F64: return launch_bp30_f64(a, s);
    case P_F32: return launch_bp30_f32(a, s);
    case P_BF16: return launch_bp30_bf16(a, s);
    case P_F16: return launch_bp30_f16(a, s);
    case P_BF16G: return launch_bp30_bf16g(a, s);
    case P_F16G: return launch_bp30_f16g(a, s);
    case P_F32G64: return launch_bp30_f32g64(a, s);
    case P_BF16G64: return launch_bp30_bf16g64(a, s);
    case P_F16G64: return launch_bp30_f16g64(a, s);
    default: return hipErrorInvalidValue;
    }
}

static constexpr std::array<int, 4> epb_table(int op, int nq) { return epb_choices(op, nq); }

int supported_epb(int op, int N, int prec, int *out, int cap)
{
    (void)prec;
    if (op < 0 || op > 2 || N < 1 || N > kMaxN) return 0;
    int cnt = 0;
    std::array<int, 4> ch{};
    switch (N + 1) {
#define FEM_CASE(q) case q: ch = epb_table(op, q); break;
        FEM_CASE(2) FEM_CASE(3) FEM_CASE(4) FEM_CASE(5) FEM_CASE(6) FEM_CASE(7) FEM_CASE(8)
        FEM_CASE(9) FEM_CASE(10) FEM_CASE(11) FEM_CASE(12) FEM_CASE(13) FEM_CASE(14)
        FEM_CASE(15) FEM_CASE(16)
#undef FEM_CASE
    default: return 0;
    }
    for (int c : ch)
        if (c > 0) {
            if (out && cnt < cap) out[cnt] = c;
            ++cnt;
        }
    return cnt;
}

int default_epb(int op, int N, int prec)
{
    (void)prec;
    // memoised like kernel_info below (the shape model is costly to evaluate)
    static std::atomic<int> memo[3][kMaxN + 1];
    if (op < 0 || op > 2 || N < 1 || N > kMaxN) return epb_default(op, N + 1);
    int v = memo[op][N].load(std::memory_order_acquire);
    if (v == 0) {
        v = epb_default(op, N + 1);
        memo[op][N].store(v, std::memory_order_release);
    }
    return v;
}

static int geo_value_bytes(int prec)
{
    switch (prec) {
    case P_F64: return 8;
    case P_F32: case P_F32G64: return 4;
    default: return 2;
    }
}

static bool kernel_info_eval(int op, int N, int prec, int epb, KernelInfo *info)
{
    int ch[kMaxEpbChoices];
    const int n = supported_epb(op, N, prec, ch, kMaxEpbChoices);
    if (epb == 0) epb = default_epb(op, N, prec);
    bool found = false;
    for (int c = 0; c < n; ++c) found |= (ch[c] == epb);
    if (!found) return false;
    const int bytes = f64_fields(prec) ? 8 : 4;   // compute type held in LDS
    info->threads = threads_for(op, N + 1, epb);
    info->lds_bytes = lds_bytes(op, N + 1, epb, bytes, geo_value_bytes(prec));
    return true;
}

// Every apply validates its launch shape, and evaluating the shape model
// (the LDS row padding simulates bank conflicts) costs about 0.1 ms on the
// host -- far more than the launch itself.  The result depends only on
// (op, N, prec, epb), so it is computed once per key and kept: 0 = not yet
// known, -1 = unsupported, else (threads << 32 | LDS bytes).  Two threads may
// both compute a key; they store the same value.
constexpr int kMemoEpb = 64;
static std::atomic<int64_t> g_kinfo[3][kMaxN + 1][P_COUNT][kMemoEpb + 1];

bool kernel_info(int op, int N, int prec, int epb, KernelInfo *info)
{
    if (op < 0 || op > 2 || N < 1 || N > kMaxN || prec < 0 || prec >= P_COUNT) return false;
    if (epb == 0) epb = default_epb(op, N, prec);
    if (epb < 1 || epb > kMemoEpb) return false;
    std::atomic<int64_t> &slot = g_kinfo[op][N][prec][epb];
    int64_t v = slot.load(std::memory_order_acquire);
    if (v == 0) {
        KernelInfo ki{};
        v = kernel_info_eval(op, N, prec, epb, &ki) ? (static_cast<int64_t>(ki.threads) << 32) | ki.lds_bytes : -1;
        slot.store(v, std::memory_order_release);
    }
    if (v < 0) return false;
    info->threads = static_cast<int>(v >> 32);
    info->lds_bytes = static_cast<int>(v & 0xFFFFFFFF);
    return true;
}

size_t cg_workspace_bytes(const fem_cg_operator *op, const fem_cg_options *opt);
int cg_solve(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x, void *ws,
             fem_cg_report *rep, hipStream_t s);

size_t assembled_workspace_bytes(const fem_cg_operator *op, const fem_assembly *as);
int assembled_apply(const fem_cg_operator *op, const fem_assembly *as, const double *ug, double *yg, void *ws,
                    hipStream_t s);
int assembled_diagonal(const fem_cg_operator *op, const fem_assembly *as, double *diag, void *ws, hipStream_t s);
int pcg_solve(const fem_cg_operator *op, const fem_assembly *as, const fem_cg_options *opt, const double *diag,
              const double *b, double *x, void *ws, fem_cg_report *rep, hipStream_t s);
hipError_t launch_gather(const int32_t *gid, const double *ug, double *ul, int64_t nl, int64_t ng, hipStream_t s);
hipError_t launch_scatter(const int32_t *off, const int32_t *loc, const double *ul, double *ug, int64_t ng,
                          int64_t nl, const double *pdot, double *part, hipStream_t s);

int check_desc(const fem_apply_desc &d);
int enqueue_desc(const fem_apply_desc &d, hipStream_t s);
double desc_bytes(const fem_apply_desc &d);
int batch_graph_create(const fem_apply_desc *d, int n, int lanes, hipStream_t s, void **graph);
int batch_graph_launch(void *graph, hipStream_t s);
int batch_graph_destroy(void *graph);

// Process-wide launch configuration: (op, N, prec) -> (epb, grid_cap).
static std::atomic<int> g_epb[3][kMaxN + 1][P_COUNT];
static std::atomic<int> g_cap[3][kMaxN + 1][P_COUNT];

}  // namespace fem

using namespace fem;

namespace {

constexpr int64_t kMaxElements = 2147483647LL;

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Bytes per value of the field vectors u and y, and of the geometric data.
size_t field_bytes(int prec) { return f64_fields(prec) ? 8 : (prec == FEM_BF16 || prec == FEM_F16) ? 2 : 4; }
size_t out_bytes(int prec) { return f64_fields(prec) ? 8 : 4; }
size_t geo_bytes(int prec)
{
    switch (prec) {
    case FEM_F64: return 8;
    case FEM_F32: case FEM_F32G64: return 4;
    default: return 2;
    }
}
bool is_f16(int prec) { return is_f16_prec(prec); }

bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + nb && pb < pa + na;
}

// FP64 fields u and y of E elements of degree N share bytes: a workgroup
// could then overwrite another element's input before that element read it.
bool fields_overlap(int N, int64_t E, const void *u, const void *y)
{
    const size_t bytes = static_cast<size_t>(E) * (N + 1) * (N + 1) * (N + 1) * sizeof(double);
    return overlap(u, bytes, y, bytes);
}

int common_checks(int op, int N, int64_t E, int prec, float geo_scale, const void *u, const void *y)
{
    if (N < 1 || N > kMaxN) return FEM_ERR_ARG;
    if (E < 0 || E > kMaxElements) return FEM_ERR_ARG;
    if (prec < 0 || prec >= P_COUNT) return FEM_ERR_UNSUPPORTED;
    if (is_f16(prec) && !(geo_scale > 0.0f)) return FEM_ERR_ARG;
    if (E == 0) return FEM_OK;
    if (!u || !y) return FEM_ERR_ARG;
    if (!aligned16(u) || !aligned16(y)) return FEM_ERR_ALIGN;
    const int64_t np = static_cast<int64_t>(N + 1) * (N + 1) * (N + 1);
    if (overlap(u, E * np * field_bytes(prec), y, E * np * out_bytes(prec))) return FEM_ERR_ARG;
    (void)op;
    return FEM_OK;
}

int tune_lookup(int op, int N, int prec, int *epb, int *cap)
{
    *epb = g_epb[op][N][prec].load(std::memory_order_relaxed);
    *cap = g_cap[op][N][prec].load(std::memory_order_relaxed);
    if (*epb == 0) *epb = default_epb(op, N, prec);
    return FEM_OK;
}

int finish(hipError_t e) { return e == hipSuccess ? FEM_OK : FEM_ERR_HIP; }

int run_apply(ApplyArgs &a, void *stream)
{
    tune_lookup(a.op, a.N, a.prec, &a.epb, &a.grid_cap);
    KernelInfo ki;
    if (!kernel_info(a.op, a.N, a.prec, a.epb, &ki)) return FEM_ERR_UNSUPPORTED;
    if (a.E == 0) return FEM_OK;
    auto s = static_cast<hipStream_t>(stream);
    switch (a.op) {
    case OP_BP10: return finish(launch_bp10(a, s));
    case OP_BP35: return finish(launch_bp35(a, s));
    case OP_BP30: return finish(launch_bp30(a, s));
    default: return FEM_ERR_UNSUPPORTED;
    }
}

bool dev_aligned(const void *p) { return aligned16(p); }

}  // namespace

namespace fem {

int check_desc(const fem_apply_desc &d)
{
    const int st = common_checks(d.op, d.N, d.E, d.prec, d.geo_scale, d.u, d.y);
    if (st != FEM_OK) return st;
    if (d.op < FEM_OP_BP10 || d.op > FEM_OP_BP30) return FEM_ERR_ARG;
    if (d.E > 0) {
        switch (d.op) {
        case FEM_OP_BP10:
            if (!d.I1d || !d.wJ) return FEM_ERR_ARG;
            if (!dev_aligned(d.wJ) || !dev_aligned(d.I1d)) return FEM_ERR_ALIGN;
            break;
        case FEM_OP_BP35:
            if (!d.D1d || !d.G || (d.lambda != 0.0 && !d.wJ)) return FEM_ERR_ARG;
            if (!dev_aligned(d.G) || !dev_aligned(d.D1d) || (d.wJ && !dev_aligned(d.wJ))) return FEM_ERR_ALIGN;
            break;
        default:
            if (!d.I1d || !d.Dgl || !d.G || (d.lambda != 0.0 && !d.wJ)) return FEM_ERR_ARG;
            if (!dev_aligned(d.G) || !dev_aligned(d.I1d) || !dev_aligned(d.Dgl) || (d.wJ && !dev_aligned(d.wJ)))
                return FEM_ERR_ALIGN;
        }
    }
    int epb, cap;
    tune_lookup(d.op, d.N, d.prec, &epb, &cap);
    KernelInfo ki;
    if (!kernel_info(d.op, d.N, d.prec, epb, &ki)) return FEM_ERR_UNSUPPORTED;
    return FEM_OK;
}

int enqueue_desc(const fem_apply_desc &d, hipStream_t s)
{
    ApplyArgs a{};
    a.op = d.op; a.N = d.N; a.E = d.E; a.I1d = d.I1d; a.D1d = d.D1d; a.Dgl = d.Dgl; a.G = d.G;
    a.wJ = d.op == FEM_OP_BP10 || d.lambda != 0.0 ? d.wJ : nullptr;
    a.u = d.u; a.y = d.y; a.lambda = d.op == FEM_OP_BP10 ? 0.0 : d.lambda; a.beta = d.beta;
    a.prec = d.prec; a.geo_scale = d.geo_scale;
    return run_apply(a, s);
}

// Algorithmic HBM bytes of one descriptor (load balancing of graph lanes).
double desc_bytes(const fem_apply_desc &d)
{
    const double nq = d.N + 1, ng = d.N + 2;
    const double np = nq * nq * nq, npg = ng * ng * ng;
    const double fb = static_cast<double>(field_bytes(d.prec)), ob = static_cast<double>(out_bytes(d.prec));
    const double gb = static_cast<double>(geo_bytes(d.prec));
    double geo;
    if (d.op == FEM_OP_BP10) geo = npg * gb;
    else if (d.op == FEM_OP_BP35) geo = (d.lambda != 0.0 ? 7.0 : 6.0) * np * gb;
    else geo = (d.lambda != 0.0 ? 7.0 : 6.0) * npg * gb;
    return static_cast<double>(d.E) * (np * (fb + ob + (d.beta != 0.0 ? ob : 0.0)) + geo);
}

}  // namespace fem

extern "C" {

const char *fem_status_str(int status)
{
    switch (status) {
    case FEM_OK: return "ok";
    case FEM_ERR_ARG: return "invalid argument";
    case FEM_ERR_UNSUPPORTED: return "unsupported configuration";
    case FEM_ERR_ALIGN: return "pointer not 16-byte aligned";
    case FEM_ERR_HIP: return "HIP runtime error";
    case FEM_ERR_NOT_CONVERGED: return "not converged";
    case FEM_ERR_BREAKDOWN: return "breakdown";
    case FEM_ERR_WORKSPACE: return "workspace too small";
    case FEM_ERR_GEOMETRY: return "non-positive Jacobian";
    default: return "unknown status";
    }
}

int fem_version(void) { return 100; }

#ifndef FEM_BUILD_ID
#define FEM_BUILD_ID "unknown"
#endif
const char *fem_build_id(void) { return FEM_BUILD_ID; }
int fem_max_degree(void) { return kMaxN; }
int64_t fem_max_elements(void) { return kMaxElements; }

int fem_basis_tables(int N, double *r_gll, double *w_gll, double *r_gl, double *w_gl, double *I1d,
                     double *D1d, double *Dgl)
{
    if (N < 1 || N > kMaxN) return FEM_ERR_ARG;
    return basis_tables(N, r_gll, w_gll, r_gl, w_gl, I1d, D1d, Dgl) ? FEM_ERR_ARG : FEM_OK;
}

int fem_geometric_factors(int N, int64_t E, int quad, const double *X, void *G, void *wJ, int prec,
                          float geo_scale, int64_t *bad_count, void *stream)
{
    if (N < 1 || N > kMaxN || E < 0 || E > kMaxElements) return FEM_ERR_ARG;
    if (quad != FEM_QUAD_GLL && quad != FEM_QUAD_GL) return FEM_ERR_ARG;
    if (prec < 0 || prec >= P_COUNT) return FEM_ERR_UNSUPPORTED;
    if (is_f16(prec) && !(geo_scale > 0.0f)) return FEM_ERR_ARG;
    if (E == 0) return FEM_OK;
    if (!X || (!G && !wJ)) return FEM_ERR_ARG;
    if (!aligned16(X) || (G && !aligned16(G)) || (wJ && !aligned16(wJ))) return FEM_ERR_ALIGN;
    if (bad_count && (reinterpret_cast<uintptr_t>(bad_count) & 7u)) return FEM_ERR_ALIGN;
    return finish(launch_geometry(N, E, quad, X, G, wJ, prec, geo_scale, bad_count,
                                  static_cast<hipStream_t>(stream)));
}

int fem_geo_vector_width(int N, int quad, int prec)
{
    if (N < 1 || N > kMaxN || (quad != FEM_QUAD_GLL && quad != FEM_QUAD_GL) || prec < 0 || prec >= P_COUNT)
        return 0;
    const int n = quad == FEM_QUAD_GLL ? N + 1 : N + 2;
    return geo_vec(n, static_cast<int>(geo_bytes(prec)));
}

int fem_node_coords(int N, int64_t E, int quad, const double *X, double *xyz, void *stream)
{
    if (N < 1 || N > kMaxN || E < 0 || E > kMaxElements) return FEM_ERR_ARG;
    if (quad != FEM_QUAD_GLL && quad != FEM_QUAD_GL) return FEM_ERR_ARG;
    if (E == 0) return FEM_OK;
    if (!X || !xyz) return FEM_ERR_ARG;
    if (!aligned16(X) || !aligned16(xyz)) return FEM_ERR_ALIGN;
    return finish(launch_node_coords(N, E, quad, X, xyz, static_cast<hipStream_t>(stream)));
}

int fem_mass_apply(int N, int64_t E, const double *I1d, const void *wJ, const void *u, void *y,
                   double beta, int prec, float geo_scale, void *stream)
{
    fem_apply_desc d{};
    d.op = FEM_OP_BP10; d.N = N; d.E = E; d.prec = prec; d.I1d = I1d; d.wJ = wJ; d.beta = beta;
    d.geo_scale = geo_scale; d.u = u; d.y = y;
    const int st = check_desc(d);
    return st != FEM_OK ? st : enqueue_desc(d, static_cast<hipStream_t>(stream));
}

int fem_stiff_collocated_apply(int N, int64_t E, const double *D1d, const void *G, const void *wJ,
                               double lambda, const void *u, void *y, double beta, int prec,
                               float geo_scale, void *stream)
{
    fem_apply_desc d{};
    d.op = FEM_OP_BP35; d.N = N; d.E = E; d.prec = prec; d.D1d = D1d; d.G = G; d.wJ = wJ;
    d.lambda = lambda; d.beta = beta; d.geo_scale = geo_scale; d.u = u; d.y = y;
    const int st = check_desc(d);
    return st != FEM_OK ? st : enqueue_desc(d, static_cast<hipStream_t>(stream));
}

int fem_stiff_collocated_vertex_apply(int N, int64_t E, const double *D1d, const double *X, double lambda,
                                      const double *u, double *y, double beta, void *stream)
{
    if (N < 1 || N > kMaxN || E < 0 || E > kMaxElements) return FEM_ERR_ARG;
    if (E == 0) return FEM_OK;
    if (!D1d || !X || !u || !y) return FEM_ERR_ARG;
    if (!aligned16(D1d) || !aligned16(X) || !aligned16(u) || !aligned16(y)) return FEM_ERR_ALIGN;
    if (fields_overlap(N, E, u, y)) return FEM_ERR_ARG;
    return finish(launch_bp35v(N, E, D1d, X, lambda, u, y, beta, 0, static_cast<hipStream_t>(stream)));
}

int fem_stiff_dealiased_vertex_apply(int N, int64_t E, const double *I1d, const double *Dgl, const double *X,
                                     double lambda, const double *u, double *y, double beta, void *stream)
{
    if (N < 1 || N > kMaxN || E < 0 || E > kMaxElements) return FEM_ERR_ARG;
    if (E == 0) return FEM_OK;
    if (!I1d || !Dgl || !X || !u || !y) return FEM_ERR_ARG;
    if (!aligned16(I1d) || !aligned16(Dgl) || !aligned16(X) || !aligned16(u) || !aligned16(y)) return FEM_ERR_ALIGN;
    if (fields_overlap(N, E, u, y)) return FEM_ERR_ARG;
    return finish(launch_bp30v(N, E, I1d, Dgl, X, lambda, u, y, beta, static_cast<hipStream_t>(stream)));
}

int fem_stiff_dealiased_apply(int N, int64_t E, const double *I1d, const double *Dgl, const void *G,
                              const void *wJ, double lambda, const void *u, void *y, double beta,
                              int prec, float geo_scale, void *stream)
{
    fem_apply_desc d{};
    d.op = FEM_OP_BP30; d.N = N; d.E = E; d.prec = prec; d.I1d = I1d; d.Dgl = Dgl; d.G = G; d.wJ = wJ;
    d.lambda = lambda; d.beta = beta; d.geo_scale = geo_scale; d.u = u; d.y = y;
    const int st = check_desc(d);
    return st != FEM_OK ? st : enqueue_desc(d, static_cast<hipStream_t>(stream));
}

int fem_batch_apply(const fem_apply_desc *d, int n, void *stream)
{
    if (n < 0 || (n > 0 && !d)) return FEM_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        const int st = check_desc(d[i]);
        if (st != FEM_OK) return st;
    }
    for (int i = 0; i < n; ++i) {
        const int st = enqueue_desc(d[i], static_cast<hipStream_t>(stream));
        if (st != FEM_OK) return st;
    }
    return FEM_OK;
}

int fem_batch_graph_create(const fem_apply_desc *d, int n, int lanes, void *stream, void **graph)
{
    if (!graph || n < 0 || (n > 0 && !d) || lanes < 1 || lanes > 8 || !stream) return FEM_ERR_ARG;
    *graph = nullptr;
    for (int i = 0; i < n; ++i) {
        const int st = check_desc(d[i]);
        if (st != FEM_OK) return st;
    }
    return batch_graph_create(d, n, lanes, static_cast<hipStream_t>(stream), graph);
}

int fem_batch_graph_launch(void *graph, void *stream)
{
    if (!graph) return FEM_ERR_ARG;
    return batch_graph_launch(graph, static_cast<hipStream_t>(stream));
}

int fem_batch_graph_destroy(void *graph)
{
    if (!graph) return FEM_ERR_ARG;
    return batch_graph_destroy(graph);
}

int fem_stream_copy(const void *src, void *dst, size_t bytes, void *stream)
{
    if (bytes == 0) return FEM_OK;
    if (!src || !dst || (bytes & 15u)) return FEM_ERR_ARG;
    if (!aligned16(src) || !aligned16(dst)) return FEM_ERR_ALIGN;
    if (overlap(src, bytes, dst, bytes)) return FEM_ERR_ARG;
    return finish(launch_copy(src, dst, bytes, static_cast<hipStream_t>(stream)));
}

int fem_lds_bandwidth(int mode, int64_t workgroups, int iters, double *sink, void *stream)
{
    if (mode < 0 || mode > 3 || workgroups < 1 || workgroups > max_grid(256) || iters < 1) return FEM_ERR_ARG;
    if (!sink) return FEM_ERR_ARG;
    if (!aligned16(sink)) return FEM_ERR_ALIGN;
    return finish(launch_lds_probe(mode, workgroups, iters, sink, static_cast<hipStream_t>(stream)));
}

static int cg_check(const fem_cg_operator *op, const fem_cg_options *opt)
{
    if (!op || !opt) return FEM_ERR_ARG;
    if (op->N < 1 || op->N > kMaxN || op->E < 0 || op->E > kMaxElements) return FEM_ERR_ARG;
    if (opt->mode < 0 || opt->mode > 2) return FEM_ERR_ARG;
    if (opt->fusion < FEM_CG_FUSE_AUTO || opt->fusion > FEM_CG_FUSE_ONEPASS) return FEM_ERR_ARG;
    if (!(opt->rtol > 0.0) || opt->max_iters < 0 || opt->delta < 0.0 || opt->delta >= 1.0 ||
        opt->check_every < 0 || opt->history_len < 0 || (opt->history_len > 0 && !opt->history))
        return FEM_ERR_ARG;
    if (op->lambda < 0.0) return FEM_ERR_ARG;
    if (op->E == 0) return FEM_OK;
    if (!op->I1d || !op->D1d || !op->G || (op->lambda != 0.0 && !op->wJ)) return FEM_ERR_ARG;
    if (!aligned16(op->G) || (op->wJ && !aligned16(op->wJ)) || !aligned16(op->I1d) || !aligned16(op->D1d))
        return FEM_ERR_ALIGN;
    if (opt->mode != 0) {
        const int p = op->inner_prec;
        if (p != FEM_F32 && p != FEM_BF16G && p != FEM_F16G && p != FEM_F32G64 && p != FEM_BF16G64 &&
            p != FEM_F16G64)
            return FEM_ERR_UNSUPPORTED;
        if (!op->G_lo || (op->lambda != 0.0 && !op->wJ_lo)) return FEM_ERR_ARG;
        if (!aligned16(op->G_lo) || (op->wJ_lo && !aligned16(op->wJ_lo))) return FEM_ERR_ALIGN;
        if (is_f16(p) && !(op->geo_scale_G > 0.0f && (op->lambda == 0.0 || op->geo_scale_wJ > 0.0f)))
            return FEM_ERR_ARG;
    }
    return FEM_OK;
}

size_t fem_cg_workspace_bytes(const fem_cg_operator *op, const fem_cg_options *opt)
{
    if (cg_check(op, opt) != FEM_OK) return 0;
    return cg_workspace_bytes(op, opt);
}

int fem_cg_solve(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x,
                 void *workspace, size_t workspace_bytes, fem_cg_report *rep, void *stream)
{
    int st = cg_check(op, opt);
    if (st != FEM_OK) return st;
    if (!rep) return FEM_ERR_ARG;
    *rep = fem_cg_report{};
    if (op->E == 0) return FEM_OK;
    if (!b || !x || !workspace) return FEM_ERR_ARG;
    if (!aligned16(b) || !aligned16(x) || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return FEM_ERR_ALIGN;
    const int64_t n = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    if (overlap(b, n * 8, x, n * 8)) return FEM_ERR_ARG;
    if (workspace_bytes < cg_workspace_bytes(op, opt)) return FEM_ERR_WORKSPACE;
    return cg_solve(op, opt, b, x, workspace, rep, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- CG without allocation
//
// fem_cg_solve_noalloc runs fem_cg_solve's code with its workspace in a
// file-scope device array: each GPU the library runs on holds one copy of
// FEM_CG_NOALLOC_BYTES bytes until the process ends.  In host code the
// array's name is a host-side stand-in, so kernels and copies get the
// device address that hipGetSymbolAddress returns, taken once per device
// with that device current (the first call on it) and kept.
static __device__ __align__(256) unsigned char scratch[FEM_CG_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

void *scratch_ptr()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

int fem_cg_solve_noalloc(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x,
                         fem_cg_report *rep, void *stream)
{
    int st = cg_check(op, opt);
    if (st != FEM_OK) return st;
    if (!rep) return FEM_ERR_ARG;
    *rep = fem_cg_report{};
    if (op->E == 0) return FEM_OK;
    if (!b || !x) return FEM_ERR_ARG;
    if (!aligned16(b) || !aligned16(x)) return FEM_ERR_ALIGN;
    const int64_t n = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    if (overlap(b, n * 8, x, n * 8)) return FEM_ERR_ARG;
    if (cg_workspace_bytes(op, opt) > static_cast<size_t>(FEM_CG_NOALLOC_BYTES)) return FEM_ERR_WORKSPACE;
    void *ws = scratch_ptr();
    if (!ws) return FEM_ERR_HIP;
    // the solve clears its own scalars; the vectors are written before they are read
    return cg_solve(op, opt, b, x, ws, rep, static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------- assembled operator

static bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
static constexpr int64_t kMaxIndex = 2147483647LL;   // int32 node numbers

int fem_assembly_inverse_map(int64_t n_local, const int32_t *gather, int64_t n_global, int32_t *offsets,
                             int32_t *locals)
{
    if (n_local < 0 || n_local > kMaxIndex || n_global < 1 || n_global > kMaxIndex) return FEM_ERR_ARG;
    if (!offsets || (n_local > 0 && (!gather || !locals))) return FEM_ERR_ARG;
    for (int64_t l = 0; l < n_local; ++l)
        if (gather[l] < 0 || gather[l] >= n_global) return FEM_ERR_ARG;
    // counting sort by global node, stable: each node's copies stay ascending
    std::memset(offsets, 0, static_cast<size_t>(n_global + 1) * sizeof(int32_t));
    for (int64_t l = 0; l < n_local; ++l) offsets[gather[l] + 1] += 1;
    for (int64_t g = 0; g < n_global; ++g) offsets[g + 1] += offsets[g];
    std::vector<int32_t> next(offsets, offsets + n_global);
    for (int64_t l = 0; l < n_local; ++l) locals[next[gather[l]]++] = static_cast<int32_t>(l);
    return FEM_OK;
}

int fem_gather(int64_t n_local, int64_t n_global, const int32_t *gather, const double *ug, double *ul,
               void *stream)
{
    if (n_local < 0 || n_local > kMaxIndex || n_global < 0 || n_global > kMaxIndex) return FEM_ERR_ARG;
    if (n_local == 0) return FEM_OK;
    if (!gather || !ug || !ul) return FEM_ERR_ARG;
    if (!aligned4(gather) || !aligned16(ug) || !aligned16(ul)) return FEM_ERR_ALIGN;
    if (overlap(ug, n_global * 8, ul, n_local * 8)) return FEM_ERR_ARG;
    return finish(launch_gather(gather, ug, ul, n_local, n_global, static_cast<hipStream_t>(stream)));
}

int fem_scatter(int64_t n_local, int64_t n_global, const int32_t *offsets, const int32_t *locals,
                const double *ul, double *ug, void *stream)
{
    if (n_local < 0 || n_local > kMaxIndex || n_global < 0 || n_global > kMaxIndex) return FEM_ERR_ARG;
    if (n_global == 0) return FEM_OK;
    if (!offsets || !locals || !ul || !ug) return FEM_ERR_ARG;
    if (!aligned4(offsets) || !aligned4(locals) || !aligned16(ug) || !aligned16(ul)) return FEM_ERR_ALIGN;
    if (overlap(ug, n_global * 8, ul, n_local * 8)) return FEM_ERR_ARG;
    return finish(launch_scatter(offsets, locals, ul, ug, n_global, n_local, nullptr, nullptr,
                                 static_cast<hipStream_t>(stream)));
}

// Operator (FP64 data only) and map of the assembled calls.
static int assembled_check(const fem_cg_operator *op, const fem_assembly *as)
{
    if (!op || !as) return FEM_ERR_ARG;
    if (op->N < 1 || op->N > kMaxN || op->E < 1 || op->lambda < 0.0) return FEM_ERR_ARG;
    const int64_t nl = op->E * static_cast<int64_t>(op->N + 1) * (op->N + 1) * (op->N + 1);
    if (nl > kMaxIndex || as->n_global < 1 || as->n_global > nl) return FEM_ERR_ARG;
    if (!op->I1d || !op->D1d || !op->G || (op->lambda != 0.0 && !op->wJ)) return FEM_ERR_ARG;
    if (!as->gather || !as->offsets || !as->locals) return FEM_ERR_ARG;
    if (!aligned16(op->G) || (op->wJ && !aligned16(op->wJ)) || !aligned16(op->I1d) || !aligned16(op->D1d))
        return FEM_ERR_ALIGN;
    if (!aligned4(as->gather) || !aligned4(as->offsets) || !aligned4(as->locals)) return FEM_ERR_ALIGN;
    return FEM_OK;
}

size_t fem_assembled_workspace_bytes(const fem_cg_operator *op, const fem_assembly *as)
{
    if (assembled_check(op, as) != FEM_OK) return 0;
    return assembled_workspace_bytes(op, as);
}

static int assembled_ws_check(const fem_cg_operator *op, const fem_assembly *as, void *ws, size_t ws_bytes)
{
    if (!ws) return FEM_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return FEM_ERR_ALIGN;
    return ws_bytes < assembled_workspace_bytes(op, as) ? FEM_ERR_WORKSPACE : FEM_OK;
}

int fem_assembled_apply(const fem_cg_operator *op, const fem_assembly *as, const double *ug, double *yg,
                        void *workspace, size_t workspace_bytes, void *stream)
{
    int st = assembled_check(op, as);
    if (st != FEM_OK) return st;
    if (!ug || !yg) return FEM_ERR_ARG;
    if (!aligned16(ug) || !aligned16(yg)) return FEM_ERR_ALIGN;
    if (overlap(ug, as->n_global * 8, yg, as->n_global * 8)) return FEM_ERR_ARG;
    if ((st = assembled_ws_check(op, as, workspace, workspace_bytes)) != FEM_OK) return st;
    return assembled_apply(op, as, ug, yg, workspace, static_cast<hipStream_t>(stream));
}

int fem_assembled_diagonal(const fem_cg_operator *op, const fem_assembly *as, double *diag, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    int st = assembled_check(op, as);
    if (st != FEM_OK) return st;
    if (!diag) return FEM_ERR_ARG;
    if (!aligned16(diag)) return FEM_ERR_ALIGN;
    if ((st = assembled_ws_check(op, as, workspace, workspace_bytes)) != FEM_OK) return st;
    return assembled_diagonal(op, as, diag, workspace, static_cast<hipStream_t>(stream));
}

int fem_pcg_solve(const fem_cg_operator *op, const fem_assembly *as, const fem_cg_options *opt, const double *diag,
                  const double *b, double *x, void *workspace, size_t workspace_bytes, fem_cg_report *rep,
                  void *stream)
{
    int st = assembled_check(op, as);
    if (st != FEM_OK) return st;
    if (!opt || !rep || opt->mode != 0) return FEM_ERR_ARG;
    if (!(opt->rtol > 0.0) || opt->max_iters < 0 || opt->check_every < 0 || opt->history_len < 0 ||
        (opt->history_len > 0 && !opt->history))
        return FEM_ERR_ARG;
    *rep = fem_cg_report{};
    if (!b || !x) return FEM_ERR_ARG;
    if (!aligned16(b) || !aligned16(x) || (diag && !aligned16(diag))) return FEM_ERR_ALIGN;
    if (overlap(b, as->n_global * 8, x, as->n_global * 8) ||
        (diag && overlap(diag, as->n_global * 8, x, as->n_global * 8)))
        return FEM_ERR_ARG;
    if ((st = assembled_ws_check(op, as, workspace, workspace_bytes)) != FEM_OK) return st;
    return pcg_solve(op, as, opt, diag, b, x, workspace, rep, static_cast<hipStream_t>(stream));
}

int fem_tune_set(int op, int N, int prec, int epb, int grid_cap)
{
    if (op < 0 || op > 2 || N < 1 || N > kMaxN || prec < 0 || prec >= P_COUNT || epb < 0 || grid_cap < 0)
        return FEM_ERR_ARG;
    if (epb != 0) {
        KernelInfo ki;
        if (!kernel_info(op, N, prec, epb, &ki)) return FEM_ERR_UNSUPPORTED;
    }
    g_epb[op][N][prec].store(epb, std::memory_order_relaxed);
    g_cap[op][N][prec].store(grid_cap, std::memory_order_relaxed);
    return FEM_OK;
}

int fem_tune_load(const char *text)
{
    if (!text) return FEM_ERR_ARG;
    struct Entry { int op, N, prec, epb, cap; };
    std::vector<Entry> entries;
    const char *line = text;
    while (*line) {
        const char *nl = std::strchr(line, '\n');
        const size_t len = nl ? static_cast<size_t>(nl - line) : std::strlen(line);
        std::string s(line, len);
        const size_t hash = s.find('#');
        if (hash != std::string::npos) s.resize(hash);
        Entry e{};
        char extra = 0;
        const int got = std::sscanf(s.c_str(), "%d %d %d %d %d %c", &e.op, &e.N, &e.prec, &e.epb, &e.cap, &extra);
        if (got == 5) {
            if (e.op < 0 || e.op > 2 || e.N < 1 || e.N > kMaxN || e.prec < 0 || e.prec >= P_COUNT ||
                e.epb < 0 || e.cap < 0)
                return FEM_ERR_ARG;
            KernelInfo ki;
            if (e.epb != 0 && !kernel_info(e.op, e.N, e.prec, e.epb, &ki)) return FEM_ERR_UNSUPPORTED;
            entries.push_back(e);
        } else if (got > 0 || s.find_first_not_of(" \t\r") != std::string::npos) {
            return FEM_ERR_ARG;
        }
        if (!nl) break;
        line = nl + 1;
    }
    for (const Entry &e : entries) {
        g_epb[e.op][e.N][e.prec].store(e.epb, std::memory_order_relaxed);
        g_cap[e.op][e.N][e.prec].store(e.cap, std::memory_order_relaxed);
    }
    return FEM_OK;
}

int fem_tune_get(int op, int N, int prec, int *epb, int *grid_cap)
{
    if (op < 0 || op > 2 || N < 1 || N > kMaxN || prec < 0 || prec >= P_COUNT || !epb || !grid_cap)
        return FEM_ERR_ARG;
    return tune_lookup(op, N, prec, epb, grid_cap);
}

int fem_kernel_info(int op, int N, int prec, int epb, int *threads, int *lds_bytes_out)
{
    if (op < 0 || op > 2 || N < 1 || N > kMaxN || prec < 0 || prec >= P_COUNT) return FEM_ERR_ARG;
    KernelInfo ki;
    if (!kernel_info(op, N, prec, epb, &ki)) return FEM_ERR_UNSUPPORTED;
    if (threads) *threads = ki.threads;
    if (lds_bytes_out) *lds_bytes_out = ki.lds_bytes;
    return FEM_OK;
}

int fem_supported_epb(int op, int N, int prec, int *epbs, int cap)
{
    if (op < 0 || op > 2 || N < 1 || N > kMaxN || prec < 0 || prec >= P_COUNT || cap < 0)
        return -FEM_ERR_ARG;
    return supported_epb(op, N, prec, epbs, cap);
}

}  // extern "C"
