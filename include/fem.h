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
 *    diagonal of J^e).
 *  - 1-D tables are FP64, row-major, in device memory: I1d[(N+2)*(N+1)]
 *    (I1d[a][i] = l_i(r~_a)), D1d[(N+1)^2] (D1d[a][i] = l_i'(r_a)),
 *    Dgl[(N+2)^2] (Dgl[a][b] = l~_b'(r~_a)).  fem_basis_tables() fills them.
 *  - Storage precision `prec` applies to u, G and wJ.  y is FP64 when
 *    prec == FEM_F64 and FP32 otherwise; reduced-precision storage computes in
 *    FP32.  FEM_F16 stores G and wJ multiplied by geo_scale (the result is
 *    divided by it), because the raw factors of fine meshes underflow FP16.
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

typedef enum { FEM_F64 = 0, FEM_F32 = 1, FEM_BF16 = 2, FEM_F16 = 3 } fem_prec;
typedef enum { FEM_OP_BP10 = 0, FEM_OP_BP35 = 1, FEM_OP_BP30 = 2 } fem_op;
typedef enum { FEM_QUAD_GLL = 0, FEM_QUAD_GL = 1 } fem_quad;

/* Human-readable name of a status code (static string). */
const char *fem_status_str(int status);

/* Library version, major*10000 + minor*100 + patch. */
int fem_version(void);

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
 * with J = dx/dr; FEM_F16 stores both times geo_scale.  If bad_count is not
 * NULL it must point to one device int64 that is incremented once per node
 * with |J| <= 0 (the caller zeroes it). */
int fem_geometric_factors(int N, int64_t E, int quad, const double *X, void *G, void *wJ,
                          int prec, float geo_scale, int64_t *bad_count, void *stream);

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

/* Launch configuration of one (operator, degree, precision): `epb` elements per
 * workgroup (0 = library default) and `grid_cap` workgroups at most (0 = one
 * workgroup per element group, no cap).  Process-wide; affects later calls. */
int fem_tune_set(int op, int N, int prec, int epb, int grid_cap);
int fem_tune_get(int op, int N, int prec, int *epb, int *grid_cap);

/* Number of threads per workgroup, LDS bytes and the supported elements-per-
 * workgroup values of one (op, N, prec) kernel family.  `epbs` receives up to
 * `cap` values; returns their count (or a negative fem_status). */
int fem_kernel_info(int op, int N, int prec, int epb, int *threads, int *lds_bytes);
int fem_supported_epb(int op, int N, int prec, int *epbs, int cap);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */
