/*
 * fem.h -- C ABI of libfem, MI355X (gfx950) tensor-product operators for
 * high-order hexahedral spectral elements.
 *
 * The operators are those of Swirydowicz, Chalmers, Karakus & Warburton,
 * "Acceleration of tensor-product operations for high-order finite element
 * methods" (arXiv 1711.00903):
 *   BP1.0  mass matrix                       M^e = I^T J^e I            (Sec. "Benchmark Problem 1", Alg. 3)
 *   BP3.5  stiffness, GLL collocation        S^e = D^T G^e D (+lambda J^e)   (Sec. "Benchmark Problem 3.5", Alg. 4)
 *   BP3.0  stiffness, GL (de-aliased)        S^e = I^T D~^T G^e D~ I (+lambda I^T J^e I)  (Sec. "BP3.0", Alg. 5)
 * The global operators are block diagonal (one block per element), so every
 * apply is element-local.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Degree 1 <= N <= 15.  Nq = N+1 GLL points and Ng = N+2 GL points per
 *    direction; Np = Nq^3, NpGL = Ng^3.
 *  - Node (i,j,k) of an element -- i along r (fastest), j along s, k along t --
 *    is stored at i + Nq*j + Nq*Nq*k; fields are [E][Np], element-major.
 *  - Geometric factors are [E][6][Npq] in the order rr, rs, rt, ss, st, tt,
 *    each already multiplied by the quadrature weights and |J| (the diagonal
 *    blocks of the matrix G^e, eq. Gdef); Npq = Np for BP3.5 (GLL nodes) and
 *    NpGL for BP3.0 (GL nodes).  Scaled Jacobians wJ are [E][Npq] (the
 *    diagonal of J^e).  Inside one element's factor block (n points per
 *    direction), node (i,j,k) sits at ((k / W) n^2 + i + n j) W + k % W:
 *    the k-values of each (i,j) column are interleaved in groups of W so that
 *    one thread loads W of them with a single 16-byte (or narrower) load.
 *    W = fem_geo_vector_width(N, quad, prec) depends on n and the storage type
 *    (W = 1 is the plain i-fastest order).  fem_geometric_factors() writes
 *    this layout.
 *  - 1-D tables are FP64, row-major, in device memory: I1d[(N+2)*(N+1)]
 *    (I1d[a][i] = l_i(r~_a)), D1d[(N+1)^2] (D1d[a][i] = l_i'(r_a)),
 *    Dgl[(N+2)^2] (Dgl[a][b] = l~_b'(r~_a)).  fem_basis_tables() fills them.
 *  - Storage precision `prec` (fem_prec) fixes the types of u, G, wJ and y:
 *        prec         u          G, wJ      y      arithmetic
 *        FEM_F64      FP64       FP64       FP64   FP64
 *        FEM_F32      FP32       FP32       FP32   FP32
 *        FEM_BF16     BF16       BF16       FP32   FP32
 *        FEM_F16      FP16       FP16       FP32   FP32
 *        FEM_BF16G    FP32       BF16       FP32   FP32
 *        FEM_F16G     FP32       FP16       FP32   FP32
 *        FEM_F32G64   FP64       FP32       FP64   FP64
 *        FEM_BF16G64  FP64       BF16       FP64   FP64
 *        FEM_F16G64   FP64       FP16       FP64   FP64
 *    The FP16 modes store G and wJ multiplied by geo_scale (> 0; the result is
 *    divided by it), because the raw factors of fine meshes underflow FP16.
 *    geo_scale is ignored by the other modes.
 *  - Every array argument is a DEVICE pointer owned by the caller, 16-byte
 *    aligned, and must stay valid until the enqueued work has finished.  The
 *    library allocates nothing inside an apply.
 *  - y <- A u + beta * y; with beta == 0, y is not read.  u and y must not
 *    overlap.
 *  - Applies are asynchronous on `stream` (a hipStream_t; NULL = the null
 *    stream).  Arguments are validated before anything is enqueued: a call that
 *    returns an error has enqueued nothing and written nothing.
 *  - Every call returns a fem_status; no exception crosses the ABI.  All calls
 *    are thread-safe.
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FEM_OK = 0,
    FEM_ERR_ARG = 1,           /* bad size, degree, NULL pointer, aliasing  */
    FEM_ERR_UNSUPPORTED = 2,   /* precision / operator / size not built     */
    FEM_ERR_ALIGN = 3,         /* a pointer is not 16-byte aligned          */
    FEM_ERR_HIP = 4,           /* the HIP runtime reported an error         */
    FEM_ERR_NOT_CONVERGED = 5,
    FEM_ERR_BREAKDOWN = 6,
    FEM_ERR_WORKSPACE = 7,
    FEM_ERR_GEOMETRY = 8       /* a node with non-positive Jacobian         */
} fem_status;

typedef enum {
    FEM_F64 = 0, FEM_F32 = 1, FEM_BF16 = 2, FEM_F16 = 3, FEM_BF16G = 4, FEM_F16G = 5,
    FEM_F32G64 = 6, FEM_BF16G64 = 7, FEM_F16G64 = 8
} fem_prec;
typedef enum { FEM_OP_BP10 = 0, FEM_OP_BP35 = 1, FEM_OP_BP30 = 2 } fem_op;
typedef enum { FEM_QUAD_GLL = 0, FEM_QUAD_GL = 1 } fem_quad;

/* Human-readable name of a status code (static string). */
const char *fem_status_str(int status);

/* Library version, major*10000 + minor*100 + patch. */
int fem_version(void);

/* Identity of the sources the library was built from: the first 16 hex
 * digits of a SHA-256 over the names and contents of the kernel and ABI
 * sources and of this header, taken at build time (static string; "unknown"
 * for a build that did not supply it).  Lets a caller detect a library that
 * is stale against its sources. */
const char *fem_build_id(void);

/* Maximum supported degree N (15). */
int fem_max_degree(void);

/* Number of elements of the largest apply (2^31 - 1). */
int64_t fem_max_elements(void);

/* HOST.  Quadrature rules and 1-D tables of degree N (Notation table;
 * eqs. interpolationOps, derivativeOps).  All pointers are host arrays:
 * r_gll, w_gll [N+1] (Gauss-Lobatto-Legendre nodes / weights, ascending),
 * r_gl, w_gl [N+2] (Gauss-Legendre), I1d [(N+2)(N+1)], D1d [(N+1)^2],
 * Dgl [(N+2)^2].  Any pointer may be NULL to skip that output.
 * FEM_ERR_ARG if N is outside [1, 15]. */
int fem_basis_tables(int N, double *r_gll, double *w_gll, double *r_gl, double *w_gl,
                     double *I1d, double *D1d, double *Dgl);

/* DEVICE.  Geometric data of trilinear hexahedra (Problem description
 * section): for each element, the map from the bi-unit cube through its 8
 * vertices X[e][a+2b+4c][0..2] (FP64, vertex (a,b,c) at r,s,t = +-1).
 * quad = FEM_QUAD_GLL evaluates at the N+1 GLL points (BP3.5), FEM_QUAD_GL at
 * the N+2 GL points (BP1.0, BP3.0).  Writes, in precision `prec`,
 *   wJ[e][n]    = w_a w_b w_c |J|                    (may be NULL)
 *   G[e][f][n]  = w_a w_b w_c |J| (J^-1 J^-T)_f       (may be NULL)
 * with J = dx/dr, in the geometry type of `prec` (see above); the FP16 modes
 * store both times geo_scale.  If bad_count is not
 * NULL it must point to one device int64 that is incremented once per node
 * with |J| <= 0 (the caller zeroes it). */
int fem_geometric_factors(int N, int64_t E, int quad, const double *X, void *G, void *wJ,
                          int prec, float geo_scale, int64_t *bad_count, void *stream);

/* Interleave width W of the geometric-data layout (see the conventions above)
 * for degree N, quadrature `quad` and precision `prec`; 0 on bad arguments. */
int fem_geo_vector_width(int N, int quad, int prec);

/* DEVICE.  Physical coordinates xyz[e][n][0..2] (FP64) of the element's tensor
 * nodes (quad as above) under the trilinear map of X. */
int fem_node_coords(int N, int64_t E, int quad, const double *X, double *xyz, void *stream);

/* DEVICE.  BP1.0 mass operator, Alg. 3 (interpolate GLL -> GL, scale by wJ,
 * project back): y = M u + beta y.  wJ at GL nodes, [E][NpGL]. */
int fem_mass_apply(int N, int64_t E, const double *I1d, const void *wJ, const void *u, void *y,
                   double beta, int prec, float geo_scale, void *stream);

/* DEVICE.  BP3.5 collocated screened-Poisson operator, Alg. 4:
 * y = (D^T G D + lambda J) u + beta y, G and wJ at GLL nodes.  wJ may be NULL
 * iff lambda == 0 (the 6-factor stiffness alone). */
int fem_stiff_collocated_apply(int N, int64_t E, const double *D1d, const void *G, const void *wJ,
                               double lambda, const void *u, void *y, double beta, int prec,
                               float geo_scale, void *stream);

/* DEVICE.  BP3.5 (Alg. 4) in FP64 with the geometric factors evaluated in the
 * kernel, per GLL point, from the element's trilinear map instead of read from
 * G and wJ: the BP3.5 optimisation section weighs loading the factors against
 * computing them from the vertices, and loads them.  Applies the same operator
 * as fem_stiff_collocated_apply with the G and wJ that fem_geometric_factors
 * (FEM_QUAD_GLL, FEM_F64) writes for X, up to rounding, while moving only the
 * fields (16 B per point instead of 64 B).
 *   y = (D^T G D + lambda J) u + beta y      (beta == 0: y is not read)
 * X[e][a+2b+4c][0..2]: the 8 vertices of element e (FP64, as for
 * fem_geometric_factors); D1d, u, y as for fem_stiff_collocated_apply with
 * prec = FEM_F64.  All are device pointers owned by the caller, 16-byte
 * aligned; u and y must not overlap.  FEM_ERR_ARG for N outside [1, 15],
 * E < 0 or beyond the element limit, a NULL pointer or overlapping u and y;
 * FEM_ERR_ALIGN for a misaligned pointer; nothing is enqueued then.
 * Asynchronous on the stream; E == 0 is a no-op. */
int fem_stiff_collocated_vertex_apply(int N, int64_t E, const double *D1d, const double *X, double lambda,
                                      const double *u, double *y, double beta, void *stream);

/* DEVICE.  BP3.0 (Alg. 5) in FP64 with the geometric factors evaluated in the
 * kernel, per Gauss point, from the element's trilinear map instead of read
 * from G and wJ (the load-or-recompute trade of the BP3.5 optimisation
 * section, for the operator whose factors are 81% of its bytes at N = 7).
 * Applies the same operator as fem_stiff_dealiased_apply with the G and wJ
 * that fem_geometric_factors (FEM_QUAD_GL, FEM_F64) writes for X, up to
 * rounding.  X as for fem_stiff_collocated_vertex_apply; I1d, Dgl, u, y as for
 * fem_stiff_dealiased_apply with prec = FEM_F64.  Device pointers owned by the
 * caller, 16-byte aligned, u and y not overlapping; errors and asynchrony as
 * for fem_stiff_collocated_vertex_apply. */
int fem_stiff_dealiased_vertex_apply(int N, int64_t E, const double *I1d, const double *Dgl, const double *X,
                                     double lambda, const double *u, double *y, double beta, void *stream);

/* DEVICE.  BP3.0 de-aliased screened-Poisson operator, Alg. 5:
 * y = I^T (D~^T G D~ + lambda J) I u + beta y, G and wJ at GL nodes.  wJ may be
 * NULL iff lambda == 0. */
int fem_stiff_dealiased_apply(int N, int64_t E, const double *I1d, const double *Dgl,
                              const void *G, const void *wJ, double lambda, const void *u, void *y,
                              double beta, int prec, float geo_scale, void *stream);

/* DEVICE.  Streaming copy of `bytes` bytes (16-byte vector loads and stores),
 * the empirical device-to-device copy roofline of the Empirical performance
 * model section (eq. globalRoof).  src and dst must not overlap; bytes must be
 * a multiple of 16. */
int fem_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* DEVICE.  LDS bandwidth probe, the measured B_sh of the shared-memory
 * roofline (Empirical performance model section, eq. sharedRoof): each of
 * `workgroups` workgroups of 256 lanes moves 256 x iters x 16 vectors through
 * its own 32 KiB of LDS, conflict-free; mode 0: 8-byte reads, 1: 16-byte
 * reads, 2: 8-byte writes, 3: 16-byte writes.  Bytes moved:
 * workgroups x 256 x iters x 16 x (8 or 16).  sink: device array of
 * workgroups x 256 doubles (the lanes' sums, so no access is dead); the
 * caller times the launch. */
int fem_lds_bandwidth(int mode, int64_t workgroups, int iters, double *sink, void *stream);

/* ---------------------------------------------------------------------------
 * Conjugate gradients on A = S + lambda M, with S the BP3.5 stiffness (GLL
 * collocation, 6 factors) and M the BP1.0 mass (GL quadrature): symmetric, and
 * positive definite for lambda > 0 (the screened Poisson operator of the
 * Problem description section, unassembled, block diagonal).
 *
 * mode 0: FP64 CG.  mode 1: mixed precision -- the Krylov iteration runs with
 * the operator's geometric data stored in `inner_prec`'s geometry type, and
 * FP32 vectors (FEM_F32, FEM_BF16G, FEM_F16G) or FP64 vectors and arithmetic
 * (FEM_F32G64, FEM_BF16G64, FEM_F16G64).  mode 2: iterative refinement -- as
 * mode 1, but every reliable update also restarts the Krylov iteration from
 * the replaced residual, so each refinement step is a fresh inner CG stopped
 * after reducing the residual by `delta`.  All modes use reliable updates: whenever the
 * recursive residual has dropped by `delta` (default 0.1) relative to the last
 * true residual, the iterate is folded into the FP64 x and r = b - A x is
 * recomputed with the FP64 operator.  The solve stops when the FP64 true
 * residual satisfies ||b - A x||_2 <= rtol ||b||_2, and reports that value.
 * The call is blocking: the host reads the residual norm every `check_every`
 * iterations (default 1).  Dot products are reduced in FP64 in a fixed order,
 * so a solve is repeatable bit for bit.
 * ------------------------------------------------------------------------- */
typedef struct {
    int N;
    int64_t E;
    const double *I1d, *D1d;   /* device tables (fem_basis_tables)                   */
    const void *G;             /* FP64 BP3.5 factors at GLL nodes, [E][6][Np]         */
    const void *wJ;            /* FP64 BP1.0 scaled Jacobians at GL nodes, [E][NpGL]; */
                               /* NULL iff lambda == 0                                */
    double lambda;
    int inner_prec;            /* mode 1: FEM_F32, FEM_BF16G, FEM_F16G, FEM_F32G64,   */
                               /* FEM_BF16G64 or FEM_F16G64                           */
    const void *G_lo, *wJ_lo;  /* mode 1: the same data in inner_prec's geometry type */
    float geo_scale_G;         /* FP16 inner mode: storage scale of G_lo              */
    float geo_scale_wJ;        /* FP16 inner mode: storage scale of wJ_lo             */
} fem_cg_operator;

/* How one Krylov iteration's p <- r + beta p, Ap = (S + lambda M) p and p . Ap
 * are split into kernels.  AUTO: two kernels where available (FP64 or FP32
 * vectors, N <= 7, lambda != 0) -- the stiffness kernel forms p as it loads it and
 * writes it back, the mass kernel adds lambda M p and emits per-element
 * partials of p . Ap -- else as NONE.  NONE: one kernel per step.  ONEPASS: a
 * single kernel for the three steps (FP64 vectors, lambda != 0, N <= 14),
 * else as NONE.  All three give the same iterates up to rounding. */
typedef enum { FEM_CG_FUSE_AUTO = 0, FEM_CG_FUSE_NONE = 1, FEM_CG_FUSE_ONEPASS = 2 } fem_cg_fusion;

typedef struct {
    int mode;                  /* 0 = FP64 CG, 1 = mixed precision, 2 = mixed         */
                               /* precision with restarts (iterative refinement)     */
    double rtol;               /* relative FP64 true-residual target                  */
    int max_iters;             /* iterations of the Krylov loop                       */
    double delta;              /* reliable-update threshold, (0, 1); 0 = 0.1          */
    int check_every;           /* host residual check period; 0 = 1                   */
    int fusion;                /* fem_cg_fusion: how the Krylov step is split into    */
                               /* kernels                                             */
    double *history;           /* HOST array or NULL: the true relative residual at   */
                               /* the start and after each reliable update           */
    int history_len;           /* capacity of history                                 */
} fem_cg_options;

typedef struct {
    int status;                /* FEM_OK, FEM_ERR_NOT_CONVERGED or FEM_ERR_BREAKDOWN  */
    int iters;                 /* Krylov iterations                                   */
    int reliable_updates;
    int hi_matvecs;            /* FP64 operator applications (true residuals)         */
    int history_count;         /* entries written to opt->history                     */
    double rel_res;            /* final ||b - A x|| / ||b||, evaluated in FP64        */
    double ms;                 /* wall time of the solve                              */
} fem_cg_report;

/* Device workspace bytes a solve needs (vectors, partial sums, scalars). */
size_t fem_cg_workspace_bytes(const fem_cg_operator *op, const fem_cg_options *opt);

/* DEVICE, blocking.  Solves A x = b: b and x are FP64 [E][Np] device vectors;
 * x holds the initial guess on entry and the solution on return.  op, opt and
 * rep are host structs.  `workspace` is a device buffer of at least
 * fem_cg_workspace_bytes() bytes (256-byte aligned), owned by the caller.
 * Returns rep->status, or FEM_ERR_ARG / FEM_ERR_WORKSPACE / FEM_ERR_HIP before
 * or during the solve. */
int fem_cg_solve(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x,
                 void *workspace, size_t workspace_bytes, fem_cg_report *rep, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops, harnesses that forbid hipMalloc): fem_cg_solve with its
 * workspace in a device array that the library holds, FEM_CG_NOALLOC_BYTES
 * bytes per GPU it runs on, from the first call on that GPU until the process
 * ends.  Arguments, results and the blocking behaviour are those of
 * fem_cg_solve.  Returns FEM_ERR_WORKSPACE, before anything is enqueued, when
 * the solve needs more than FEM_CG_NOALLOC_BYTES (fem_cg_workspace_bytes);
 * with FP64 vectors that is about 48 bytes per DOF, so up to ~1.4M DOFs
 * (E = 2730 at N = 7).  The call allocates nothing.  Every call on one GPU
 * shares that GPU's array and leaves its contents behind (a solve initialises
 * what it reads): calls that overlap in time on one GPU, from several host
 * threads or on several streams, race and give wrong results.  The stream
 * must belong to the current device. */
#define FEM_CG_NOALLOC_BYTES (64u << 20)
int fem_cg_solve_noalloc(const fem_cg_operator *op, const fem_cg_options *opt, const double *b, double *x,
                         fem_cg_report *rep, void *stream);

/* ---------------------------------------------------------------------------
 * Assembled (continuous) operator.  The applies above act on each element's
 * own copy of its nodes: one block-diagonal matrix (Problem description
 * section).  On a conforming mesh neighbouring elements share the nodes of
 * their common faces, edges and corners; with Z the Boolean map that copies
 * global node values to the element-local nodes, the global finite-element
 * operator is A = Z^T A_L Z.  Z is given by `gather` ([E][Np], int32: the
 * global node of each local node, element-major, local node order as for the
 * fields); Z^T by its inverse, `offsets` ([n_global + 1]) and `locals`
 * ([E Np]): the local copies of global node g are locals[offsets[g] ..
 * offsets[g+1] - 1], in ascending order (fem_assembly_inverse_map builds
 * them).  Z^T sums each node's copies in that order, so results are
 * repeatable bit for bit.  Index maps are read on the device with every
 * index checked against its range (an entry out of range reads as zero):
 * a wrong map gives wrong values, never an access outside the arrays.
 * Limits: E Np and n_global below 2^31.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n_global;          /* number of global nodes                              */
    const int32_t *gather;     /* [E][Np] device: global node of each local node      */
    const int32_t *offsets;    /* [n_global + 1] device                               */
    const int32_t *locals;     /* [E Np] device: local nodes grouped by global node   */
} fem_assembly;

/* HOST.  The inverse map of a gather map: offsets [n_global + 1] and locals
 * [n_local] (host arrays) from gather [n_local] (host).  FEM_ERR_ARG if an
 * entry of gather lies outside [0, n_global) or a size is out of range. */
int fem_assembly_inverse_map(int64_t n_local, const int32_t *gather, int64_t n_global, int32_t *offsets,
                             int32_t *locals);

/* DEVICE.  ul = Z ug: ul[l] = ug[gather[l]], l < n_local. */
int fem_gather(int64_t n_local, int64_t n_global, const int32_t *gather, const double *ug, double *ul,
               void *stream);

/* DEVICE.  ug = Z^T ul: ug[g] = sum of ul[locals[k]], offsets[g] <= k < offsets[g+1]. */
int fem_scatter(int64_t n_local, int64_t n_global, const int32_t *offsets, const int32_t *locals,
                const double *ul, double *ug, void *stream);

/* Device workspace bytes of fem_assembled_apply, fem_assembled_diagonal and
 * fem_pcg_solve for this operator and map (two local and four global
 * vectors, partial sums); 0 on invalid arguments. */
size_t fem_assembled_workspace_bytes(const fem_cg_operator *op, const fem_assembly *as);

/* DEVICE.  yg = Z^T (S + lambda M) Z ug, the FP64 operator of fem_cg_solve
 * (op->G, op->wJ; the narrow fields of op are ignored) assembled over the
 * shared nodes.  ug, yg: [n_global] FP64, not overlapping.  workspace: device,
 * 256-byte aligned, at least fem_assembled_workspace_bytes(). */
int fem_assembled_apply(const fem_cg_operator *op, const fem_assembly *as, const double *ug, double *yg,
                        void *workspace, size_t workspace_bytes, void *stream);

/* DEVICE.  diag[n_global] = the diagonal of Z^T (S + lambda M) Z, i.e. Z^T of
 * each element's diagonal (the Jacobi preconditioner of fem_pcg_solve). */
int fem_assembled_diagonal(const fem_cg_operator *op, const fem_assembly *as, double *diag, void *workspace,
                           size_t workspace_bytes, void *stream);

/* DEVICE, blocking.  Preconditioned CG on the assembled system
 * Z^T (S + lambda M) Z x = b, FP64 throughout (opt->mode must be 0; fusion is
 * ignored), with the Jacobi preconditioner z = r / diag (diag as written by
 * fem_assembled_diagonal; NULL: no preconditioner).  b, x: [n_global] FP64;
 * x holds the initial guess on entry.  The solve stops when the FP64 true
 * residual ||b - A x|| <= rtol ||b||; when the recursive residual meets the
 * target first, the true residual is checked and, if it does not, the
 * iteration restarts from it (rep->reliable_updates counts the checks,
 * opt->history receives the true relative residuals).  Returns rep->status as
 * fem_cg_solve does. */
int fem_pcg_solve(const fem_cg_operator *op, const fem_assembly *as, const fem_cg_options *opt, const double *diag,
                  const double *b, double *x, void *workspace, size_t workspace_bytes, fem_cg_report *rep,
                  void *stream);

/* ---------------------------------------------------------------------------
 * Ragged batches: independent applies of different meshes, degrees,
 * operators and precisions (each descriptor is one fem_*_apply call; I1d is
 * used by BP1.0 and BP3.0, D1d by BP3.5, Dgl by BP3.0; wJ may be NULL where the
 * single call allows it).  All descriptors are validated before anything is
 * enqueued.
 * ------------------------------------------------------------------------- */
typedef struct {
    int op;                    /* fem_op                                              */
    int N;
    int64_t E;
    int prec;                  /* fem_prec                                            */
    const double *I1d, *D1d, *Dgl;
    const void *G, *wJ;
    double lambda, beta;
    float geo_scale;
    const void *u;
    void *y;
} fem_apply_desc;

/* DEVICE.  Enqueues the n applies on `stream` in order. */
int fem_batch_apply(const fem_apply_desc *d, int n, void *stream);

/* Captures the n applies into a HIP graph: they are spread over `lanes`
 * (1..8) forked streams, largest first, so independent meshes may run
 * concurrently, and joined back into `stream`.  *graph receives an opaque
 * handle owning the graph, its executable and the forked streams.  The
 * descriptors' buffers must stay valid until fem_batch_graph_destroy. */
int fem_batch_graph_create(const fem_apply_desc *d, int n, int lanes, void *stream, void **graph);

/* DEVICE.  One replay of the captured batch on `stream`. */
int fem_batch_graph_launch(void *graph, void *stream);

/* Releases the graph and everything it owns (synchronises its streams). */
int fem_batch_graph_destroy(void *graph);

/* Launch configuration of one (operator, degree, precision): `epb` elements per
 * workgroup (0 = library default) and `grid_cap` workgroups at most (0 = one
 * workgroup per element group, no cap).  Process-wide; affects later calls. */
int fem_tune_set(int op, int N, int prec, int epb, int grid_cap);
int fem_tune_get(int op, int N, int prec, int *epb, int *grid_cap);

/* Number of threads per workgroup, LDS bytes and the supported elements-per-
 * workgroup values of one (op, N, prec) kernel family.  `epbs` receives up to
 * `cap` values; returns their count (or a negative fem_status). */
int fem_kernel_info(int op, int N, int prec, int epb, int *threads, int *lds_bytes);

/* Loads a tune table from text: one entry per line, "op N prec epb grid_cap"
 * (integers; '#' starts a comment).  Entries are validated like
 * fem_tune_set; on the first bad line nothing is applied and FEM_ERR_ARG or
 * FEM_ERR_UNSUPPORTED is returned. */
int fem_tune_load(const char *text);
int fem_supported_epb(int op, int N, int prec, int *epbs, int cap);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */
