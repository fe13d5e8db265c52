// launch.hpp -- host-side interface between the C ABI (fem_api.cpp) and the
// kernel translation units.  Plain structs of device pointers and scalars.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace fem {

enum Prec {
    P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_F16 = 3, P_BF16G = 4, P_F16G = 5,
    P_F32G64 = 6, P_BF16G64 = 7, P_F16G64 = 8, P_COUNT = 9
};
constexpr bool is_f16_prec(int p) { return p == P_F16 || p == P_F16G || p == P_F16G64; }
// FP64 fields (and FP64 arithmetic) in these modes
constexpr bool f64_fields(int p) { return p == P_F64 || p == P_F32G64 || p == P_BF16G64 || p == P_F16G64; }
enum Op { OP_BP10 = 0, OP_BP35 = 1, OP_BP30 = 2 };

constexpr int kMaxN = 15;
constexpr int kMaxEpbChoices = 4;

// A dispatch counts its work-items in 32 bits (grid x workgroup size < 2^32)
// and its workgroups below 2^31.  Largest number of `threads`-thread
// workgroups one launch may have; element kernels with more element groups
// than that loop over them (persistent form) or split the elements over
// several launches.
constexpr int64_t max_grid(int threads)
{
    const int64_t g = 0xFFFFFFFFLL / threads;
    return g < 0x7FFFFFFFLL ? g : 0x7FFFFFFFLL;
}

struct ApplyArgs {
    int op;
    int N;
    int64_t E;
    const double *I1d;   // (N+2) x (N+1)
    const double *D1d;   // (N+1) x (N+1)
    const double *Dgl;   // (N+2) x (N+2)
    const void *G;       // [E][6][Npq]
    const void *wJ;      // [E][Npq] or null
    const void *u;       // [E][Np]
    void *y;             // [E][Np]
    double lambda;
    double beta;
    double out_scale = 1.0;   // y = out_scale * (A u) + beta y (FP16 modes also divide by geo_scale)
    float geo_scale;
    int prec;
    int epb;             // elements per workgroup, 0 = default
    int grid_cap;        // max workgroups, 0 = uncapped
    // Conjugate-gradient extensions (FP64 or FP32 fields; xr has the fields'
    // type).  BP3.5 with xr set first replaces u in place by xr + (*xbeta) u
    // (the direction update) and applies the operator to the result.  BP1.0
    // (one-wave kernel) with part set writes part[e] = sum over element e's
    // nodes of u * y (products and sum in FP64), y the final output.
    const void *xr = nullptr;
    const double *xbeta = nullptr;
    // With xr and xl set, BP3.5 also adds (*xalpha) u (u before the direction
    // update) into xl: the iterate update of the previous Krylov step.
    void *xl = nullptr;
    const double *xalpha = nullptr;
    double *part = nullptr;
};

struct KernelInfo {
    int threads;
    int lds_bytes;
};

// Each returns a hipError_t from the launch (hipSuccess when enqueued).
hipError_t launch_bp35(const ApplyArgs &a, hipStream_t s);
hipError_t launch_bp10(const ApplyArgs &a, hipStream_t s);
hipError_t launch_bp30(const ApplyArgs &a, hipStream_t s);

// Supported elements-per-workgroup values of (op, N, prec); returns count.
int supported_epb(int op, int N, int prec, int *out, int cap);
int default_epb(int op, int N, int prec);
bool kernel_info(int op, int N, int prec, int epb, KernelInfo *info);

hipError_t launch_geometry(int N, int64_t E, int quad, const double *X, void *G, void *wJ,
                           int prec, float geo_scale, int64_t *bad, hipStream_t s);
hipError_t launch_node_coords(int N, int64_t E, int quad, const double *X, double *xyz,
                              hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_lds_probe(int mode, int64_t workgroups, int iters, double *sink, hipStream_t s);

// Host-side quadrature and tables (basis.cpp).
int basis_tables(int N, double *r_gll, double *w_gll, double *r_gl, double *w_gl, double *I1d,
                 double *D1d, double *Dgl);
int gauss_lobatto(int N, double *r, double *w);
int gauss_legendre(int n, double *r, double *w);

}  // namespace fem
