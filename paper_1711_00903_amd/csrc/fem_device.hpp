// fem_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// storage types and conversions, the column/slab thread layout, and the
// launch-shape helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace fem {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Storage types.  Fields (u, y) are FP64, FP32, BF16 or FP16, and geometric
// data (G, wJ) FP64, FP32, BF16 or FP16; the arithmetic type follows from the
// pair (compute_pair below).
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
using f16_t = _Float16;

// Arithmetic type of a kernel with geometric data TG and fields TV: FP64 as
// soon as the fields are FP64 (rounding the fields to FP32 would swamp the
// smallest modes of ill-conditioned operators), FP32 otherwise.
template <class TG, class TV> struct compute_pair {
    using type = typename std::conditional<std::is_same<TG, double>::value ||
                                               std::is_same<TV, double>::value,
                                           double, float>::type;
};

template <class T> struct output_of { using type = float; };
template <> struct output_of<double> { using type = double; };

__device__ __forceinline__ double to_compute(double v, double) { return v; }
__device__ __forceinline__ float to_compute(float v, float) { return v; }
__device__ __forceinline__ float to_compute(bf16_t v, float)
{
    return __uint_as_float(static_cast<uint32_t>(v.bits) << 16);
}
__device__ __forceinline__ float to_compute(f16_t v, float) { return static_cast<float>(v); }
__device__ __forceinline__ double to_compute(float v, double) { return v; }
__device__ __forceinline__ double to_compute(bf16_t v, double) { return to_compute(v, 0.0f); }
__device__ __forceinline__ double to_compute(f16_t v, double) { return static_cast<float>(v); }

template <class TC, class TS>
__device__ __forceinline__ TC ld(const TS *__restrict__ p, int64_t idx)
{
    return to_compute(p[idx], TC{});
}

// Round-to-nearest-even float -> bfloat16 (finite inputs).
__device__ __forceinline__ bf16_t to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return bf16_t{static_cast<uint16_t>(u >> 16)};
}

template <class TS> __device__ __forceinline__ TS from_double(double v);
template <> __device__ __forceinline__ double from_double<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_double<float>(double v) { return static_cast<float>(v); }
template <> __device__ __forceinline__ bf16_t from_double<bf16_t>(double v) { return to_bf16(static_cast<float>(v)); }
// FP16 storage rounds in two steps, FP64 -> FP32 -> FP16 (each to nearest
// even), as BF16 does.  The empty asm keeps the compiler from merging the two
// conversions into one FP64 -> FP16 rounding, which differs from the two-step
// result wherever the FP32 value falls exactly halfway between two FP16 values.
template <> __device__ __forceinline__ f16_t from_double<f16_t>(double v)
{
    float f = static_cast<float>(v);
    asm volatile("" : "+v"(f));
    return static_cast<f16_t>(f);
}

// Non-temporal load for data that is streamed exactly once (geometric factors):
// keeps them from evicting the field vectors from the caches.
__device__ __forceinline__ double nt_load(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float nt_load(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ bf16_t nt_load(const bf16_t *p)
{
    return bf16_t{__builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p))};
}
__device__ __forceinline__ f16_t nt_load(const f16_t *p) { return __builtin_nontemporal_load(p); }

template <class TC, class TS>
__device__ __forceinline__ TC ld_stream(const TS *__restrict__ p, int64_t idx)
{
    return to_compute(nt_load(p + idx), TC{});
}

// ---------------------------------------------------------------------------
// Layout of geometric data (G factors and scaled Jacobians) inside one element.
// For a tensor grid of n points per direction, node (i,j,k) -- column
// col = i + n j -- of one factor block sits at
//     ((k / W) n^2 + col) W + k % W,
// i.e. the k-values of a column are interleaved in groups of W, so the thread
// that owns the column loads W of its slabs with one vector load, and the 64
// lanes of a wave read 64 W consecutive values.  W is the largest power of two
// that divides n with W values in at most 16 bytes; W = 1 is the plain
// i-fastest order.
// ---------------------------------------------------------------------------
constexpr int geo_vec(int n, int bytes)
{
    int w = 16 / bytes;
    while (w > 1 && n % w) w >>= 1;
    return w;
}

__host__ __device__ constexpr int64_t geo_offset(int col, int k, int n, int W)
{
    return (static_cast<int64_t>(k / W) * n * n + col) * W + k % W;
}

template <int BYTES> struct raw_vec;
template <> struct raw_vec<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };
template <> struct raw_vec<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct raw_vec<4> { typedef unsigned int type; };
template <> struct raw_vec<2> { typedef unsigned short type; };

// One aligned vector of W stored values, kept packed in registers (a 16-bit
// or FP32 value takes a half or one VGPR instead of the two of its FP64
// widening) and widened to the compute type only when used.
template <int W, class TS> struct packed_vec {
    using R = typename raw_vec<W * sizeof(TS)>::type;
    R v;
    __device__ __forceinline__ void stream(const TS *__restrict__ p)
    {
        v = __builtin_nontemporal_load(reinterpret_cast<const R *>(p));
    }
    __device__ __forceinline__ void load(const TS *__restrict__ p) { v = *reinterpret_cast<const R *>(p); }
    __device__ __forceinline__ void zero() { v = R{}; }
    template <class TC> __device__ __forceinline__ TC get(int r) const
    {
        TS tmp[W];
        __builtin_memcpy(tmp, &v, sizeof(R));
        return to_compute(tmp[r], TC{});
    }
};

// W consecutive stored values (one aligned vector), loaded and converted to
// the compute type.
template <int W, class TC, class TS>
__device__ __forceinline__ void ld_vec(const TS *__restrict__ p, TC *out)
{
    using R = typename raw_vec<W * sizeof(TS)>::type;
    const R v = *reinterpret_cast<const R *>(p);
    TS tmp[W];
    __builtin_memcpy(tmp, &v, sizeof(R));
#pragma unroll
    for (int r = 0; r < W; ++r) out[r] = to_compute(tmp[r], TC{});
}

// W consecutive stored values (one aligned vector), streamed non-temporally and
// converted to the compute type.
template <int W, class TC, class TS>
__device__ __forceinline__ void ld_stream_vec(const TS *__restrict__ p, TC *out)
{
    using R = typename raw_vec<W * sizeof(TS)>::type;
    const R v = __builtin_nontemporal_load(reinterpret_cast<const R *>(p));
    TS tmp[W];
    __builtin_memcpy(tmp, &v, sizeof(R));
#pragma unroll
    for (int r = 0; r < W; ++r) out[r] = to_compute(tmp[r], TC{});
}

// ---------------------------------------------------------------------------
// Launch shapes.
// ---------------------------------------------------------------------------
constexpr int round_up_wave(int n) { return (n + kWave - 1) / kWave * kWave; }

// Row length (in values) of an LDS slab whose rows hold `n` values of `bytes`
// bytes.  A thread reads a whole row with the widest aligned LDS reads, and the
// lanes of a wave read up to n different rows at once: pick the smallest
// padded length (kept 16-byte aligned for even n) for which those rows start
// in disjoint groups of the 64 four-byte banks.
constexpr int bank_conflicts(int P, int n, int bytes)
{
    const int words = P * bytes / 4;
    const int width = (n * bytes % 16 == 0) ? 4 : (bytes >= 8 ? 2 : 1);
    int worst = 0;
    for (int b = 0; b < 64; ++b) {
        int hits = 0;
        for (int r = 0; r < n && r < 64; ++r) {
            int start = (r * words) % 64;
            for (int x = 0; x < width; ++x)
                if ((start + x) % 64 == b) ++hits;
        }
        if (hits > worst) worst = hits;
    }
    return worst;
}

constexpr int lds_row(int n, int bytes)
{
    int best = n, best_c = bank_conflicts(n, n, bytes);
    const int step = (n * bytes % 16 == 0) ? 16 / bytes : 1;
    for (int P = n + step; P <= n + 4 * step; P += step) {
        int c = bank_conflicts(P, n, bytes);
        if (c < best_c) { best = P; best_c = c; }
    }
    return best;
}

// One table (row-major rows x cols of FP64 in global memory) staged in LDS in
// the compute precision.
template <class TC>
__device__ __forceinline__ void stage_table(TC *__restrict__ dst, const double *__restrict__ src,
                                            int count)
{
    for (int t = threadIdx.x; t < count; t += blockDim.x) dst[t] = static_cast<TC>(src[t]);
}

}  // namespace fem
