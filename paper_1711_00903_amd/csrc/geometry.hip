// geometry.hip -- set-up kernels: geometric factors and node coordinates of
// trilinear hexahedra (Problem description section), and the streaming copy
// that calibrates the empirical bandwidth roofline (Empirical performance
// model section, eq. globalRoof).
//
// Geometry.  Vertex v = a + 2b + 4c sits at reference corner
// (xi, eta, zeta) = (2a-1, 2b-1, 2c-1); the trilinear map is
//   x(r,s,t) = 1/8 sum_v X_v (1 + xi_v r)(1 + eta_v s)(1 + zeta_v t).
// With the covariant vectors a_r = dx/dr, a_s = dx/ds, a_t = dx/dt,
//   |J| = a_r . (a_s x a_t),
// and the contravariant vectors grad r = (a_s x a_t)/|J|, grad s = (a_t x a_r)/|J|,
// grad t = (a_r x a_s)/|J|.  The weighted metric is therefore
//   G_ab = w |J| grad r_a . grad r_b = w (c_a . c_b) / |J|,
// with c_r = a_s x a_t, c_s = a_t x a_r, c_t = a_r x a_s.
#include "fem_device.hpp"
#include "launch.hpp"

namespace fem {

struct NodeRule {
    double r[kMaxN + 2];
    double w[kMaxN + 2];
};

struct Vec3 {
    double x, y, z;
};
__device__ __forceinline__ Vec3 cross(const Vec3 &p, const Vec3 &q)
{
    return {p.y * q.z - p.z * q.y, p.z * q.x - p.x * q.z, p.x * q.y - p.y * q.x};
}
__device__ __forceinline__ double dot(const Vec3 &p, const Vec3 &q)
{
    return p.x * q.x + p.y * q.y + p.z * q.z;
}

template <class TS>
__global__ __launch_bounds__(256) void geometry_kernel(int nq, int64_t E, const double *__restrict__ X,
                                                       NodeRule rule, TS *__restrict__ G,
                                                       TS *__restrict__ wJ, double scale,
                                                       int64_t *__restrict__ bad)
{
    const int64_t npq = static_cast<int64_t>(nq) * nq * nq;
    const int64_t total = E * npq;
    const int vw = geo_vec(nq, sizeof(TS));
    for (int64_t id = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; id < total;
         id += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = id / npq;
        const int n = static_cast<int>(id - e * npq);
        const int a = n % nq, b = (n / nq) % nq, c = n / (nq * nq);
        const double r = rule.r[a], s = rule.r[b], t = rule.r[c];
        const double *Xe = X + 24 * e;
        Vec3 ar{0, 0, 0}, as{0, 0, 0}, at{0, 0, 0};
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const double xi = (v & 1) ? 1.0 : -1.0;
            const double eta = (v & 2) ? 1.0 : -1.0;
            const double zeta = (v & 4) ? 1.0 : -1.0;
            const double fr = 0.125 * xi * (1.0 + eta * s) * (1.0 + zeta * t);
            const double fs = 0.125 * eta * (1.0 + xi * r) * (1.0 + zeta * t);
            const double ft = 0.125 * zeta * (1.0 + xi * r) * (1.0 + eta * s);
            const double px = Xe[3 * v], py = Xe[3 * v + 1], pz = Xe[3 * v + 2];
            ar.x += fr * px; ar.y += fr * py; ar.z += fr * pz;
            as.x += fs * px; as.y += fs * py; as.z += fs * pz;
            at.x += ft * px; at.y += ft * py; at.z += ft * pz;
        }
        const Vec3 cr = cross(as, at), cs = cross(at, ar), ct = cross(ar, as);
        const double det = dot(ar, cr);
        if (!(det > 0.0) && bad) atomicAdd(reinterpret_cast<unsigned long long *>(bad), 1ull);
        const double w = rule.w[a] * rule.w[b] * rule.w[c];
        const int64_t off = geo_offset(a + nq * b, c, nq, vw);
        if (wJ) wJ[e * npq + off] = from_double<TS>(scale * w * det);
        if (G) {
            const double f = scale * w / det;
            TS *Ge = G + e * 6 * npq + off;
            Ge[0 * npq] = from_double<TS>(f * dot(cr, cr));
            Ge[1 * npq] = from_double<TS>(f * dot(cr, cs));
            Ge[2 * npq] = from_double<TS>(f * dot(cr, ct));
            Ge[3 * npq] = from_double<TS>(f * dot(cs, cs));
            Ge[4 * npq] = from_double<TS>(f * dot(cs, ct));
            Ge[5 * npq] = from_double<TS>(f * dot(ct, ct));
        }
    }
}

__global__ __launch_bounds__(256) void node_coords_kernel(int nq, int64_t E, const double *__restrict__ X,
                                                          NodeRule rule, double *__restrict__ xyz)
{
    const int64_t npq = static_cast<int64_t>(nq) * nq * nq;
    const int64_t total = E * npq;
    for (int64_t id = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; id < total;
         id += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t e = id / npq;
        const int n = static_cast<int>(id - e * npq);
        const int a = n % nq, b = (n / nq) % nq, c = n / (nq * nq);
        const double r = rule.r[a], s = rule.r[b], t = rule.r[c];
        const double *Xe = X + 24 * e;
        double x = 0, y = 0, z = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const double f = 0.125 * (1.0 + ((v & 1) ? r : -r)) * (1.0 + ((v & 2) ? s : -s)) *
                             (1.0 + ((v & 4) ? t : -t));
            x += f * Xe[3 * v];
            y += f * Xe[3 * v + 1];
            z += f * Xe[3 * v + 2];
        }
        xyz[3 * id] = x;
        xyz[3 * id + 1] = y;
        xyz[3 * id + 2] = z;
    }
}

static NodeRule make_rule(int N, int quad)
{
    NodeRule rule{};
    if (quad == 0) gauss_lobatto(N, rule.r, rule.w);
    else gauss_legendre(N + 2, rule.r, rule.w);
    return rule;
}

static unsigned grid_for(int64_t total, int threads)
{
    int64_t blocks = (total + threads - 1) / threads;
    const int64_t cap = 256 * 64;   // 64 workgroups per CU is plenty for set-up work
    if (blocks > cap) blocks = cap;
    return static_cast<unsigned>(blocks < 1 ? 1 : blocks);
}

hipError_t launch_geometry(int N, int64_t E, int quad, const double *X, void *G, void *wJ, int prec,
                           float geo_scale, int64_t *bad, hipStream_t s)
{
    const int nq = quad == 0 ? N + 1 : N + 2;
    const int64_t total = E * nq * nq * nq;
    if (total == 0) return hipSuccess;
    const NodeRule rule = make_rule(N, quad);
    const double scale = is_f16_prec(prec) ? static_cast<double>(geo_scale) : 1.0;
    const unsigned grid = grid_for(total, 256);
    switch (prec) {
    case P_F64:
        hipLaunchKernelGGL(geometry_kernel<double>, dim3(grid), dim3(256), 0, s, nq, E, X, rule,
                           static_cast<double *>(G), static_cast<double *>(wJ), scale, bad);
        break;
    case P_F32:
    case P_F32G64:
        hipLaunchKernelGGL(geometry_kernel<float>, dim3(grid), dim3(256), 0, s, nq, E, X, rule,
                           static_cast<float *>(G), static_cast<float *>(wJ), scale, bad);
        break;
    case P_BF16:
    case P_BF16G:
    case P_BF16G64:
        hipLaunchKernelGGL(geometry_kernel<bf16_t>, dim3(grid), dim3(256), 0, s, nq, E, X, rule,
                           static_cast<bf16_t *>(G), static_cast<bf16_t *>(wJ), scale, bad);
        break;
    case P_F16:
    case P_F16G:
    case P_F16G64:
        hipLaunchKernelGGL(geometry_kernel<f16_t>, dim3(grid), dim3(256), 0, s, nq, E, X, rule,
                           static_cast<f16_t *>(G), static_cast<f16_t *>(wJ), scale, bad);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_node_coords(int N, int64_t E, int quad, const double *X, double *xyz, hipStream_t s)
{
    const int nq = quad == 0 ? N + 1 : N + 2;
    const int64_t total = E * nq * nq * nq;
    if (total == 0) return hipSuccess;
    const NodeRule rule = make_rule(N, quad);
    hipLaunchKernelGGL(node_coords_kernel, dim3(grid_for(total, 256)), dim3(256), 0, s, nq, E, X,
                       rule, xyz);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming copy: one workgroup per 16 KiB chunk (256 threads x 4 x 16-byte
// vectors), all four loads issued before the stores.  A non-persistent grid of
// small chunks keeps every CU's queue full and reaches a higher HBM rate on
// gfx950 than a grid-stride loop over a fixed grid.
// ---------------------------------------------------------------------------
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyUnroll = 4;
constexpr int kCopyThreads = 256;

__global__ __launch_bounds__(kCopyThreads) void copy_kernel(const u32x4 *__restrict__ src,
                                                            u32x4 *__restrict__ dst, int64_t n)
{
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kCopyThreads * kCopyUnroll) + threadIdx.x;
    u32x4 v[kCopyUnroll];
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const int64_t i = base + k * kCopyThreads;
        if (i < n) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kCopyUnroll; ++k) {
        const int64_t i = base + k * kCopyThreads;
        if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const int64_t n = static_cast<int64_t>(bytes / 16);
    if (n == 0) return hipSuccess;
    const int64_t per = kCopyThreads * kCopyUnroll;
    // launches of at most max_grid workgroups, each over its own piece
    const int64_t piece = max_grid(kCopyThreads) * per;
    for (int64_t v0 = 0; v0 < n; v0 += piece) {
        const int64_t m = n - v0 < piece ? n - v0 : piece;
        hipLaunchKernelGGL(copy_kernel, dim3(static_cast<unsigned>((m + per - 1) / per)), dim3(kCopyThreads), 0, s,
                           static_cast<const u32x4 *>(src) + v0, static_cast<u32x4 *>(dst) + v0, m);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LDS bandwidth probe: the shared-memory term of the empirical performance
// model (Empirical performance model section, eq. sharedRoof), measured
// rather than taken from a data sheet.  Each workgroup of kLdsThreads lanes
// owns a 32 KiB LDS buffer; every lane reads (or writes) `iters` x kLdsUnroll
// distinct vectors of `W` doubles, lane-consecutive (a wave touches a
// contiguous 64 W x 8-byte span: no bank conflicts), so the LDS moves
// workgroups x kLdsThreads x iters x kLdsUnroll x 8 W bytes.  The result is
// summed into sink[] so that no access is dead.
// ---------------------------------------------------------------------------
constexpr int kLdsThreads = 256;
constexpr int kLdsUnroll = 16;
constexpr int kLdsValues = 4096;   // doubles per workgroup buffer (32 KiB)

template <int W, bool WRITE>
__global__ __launch_bounds__(kLdsThreads) void lds_probe_kernel(int iters, double *__restrict__ sink)
{
    typedef double vec __attribute__((ext_vector_type(W)));
    __shared__ __align__(16) double buf[kLdsValues];
    const int t = threadIdx.x;
    for (int q = t; q < kLdsValues; q += kLdsThreads) buf[q] = static_cast<double>(q);
    __syncthreads();
    vec *v = reinterpret_cast<vec *>(buf);
    constexpr int nvec = kLdsValues / W;
    constexpr int stride = nvec / kLdsUnroll;   // a lane's kLdsUnroll accesses of one pass are distinct
    vec acc = vec(0.0);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kLdsUnroll; ++u) {
            const int idx = (t + stride * u + it * 7) & (nvec - 1);
            if (WRITE) {
                v[idx] = acc + static_cast<double>(u);
                __asm__ volatile("" ::: "memory");   // keep every store (no merging across the loop)
            } else {
                acc += v[idx];
            }
        }
        if (WRITE) acc += 1.0;
    }
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += acc[w];
    if (WRITE) s += buf[t];
    sink[static_cast<int64_t>(blockIdx.x) * kLdsThreads + t] = s;
}

hipError_t launch_lds_probe(int mode, int64_t workgroups, int iters, double *sink, hipStream_t s)
{
    const dim3 grid(static_cast<unsigned>(workgroups)), block(kLdsThreads);
    switch (mode) {
    case 0: hipLaunchKernelGGL((lds_probe_kernel<1, false>), grid, block, 0, s, iters, sink); break;
    case 1: hipLaunchKernelGGL((lds_probe_kernel<2, false>), grid, block, 0, s, iters, sink); break;
    case 2: hipLaunchKernelGGL((lds_probe_kernel<1, true>), grid, block, 0, s, iters, sink); break;
    case 3: hipLaunchKernelGGL((lds_probe_kernel<2, true>), grid, block, 0, s, iters, sink); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fem
