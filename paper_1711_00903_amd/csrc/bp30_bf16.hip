// BP3.0 kernels: geometric data stored as bf16_t, fields as bf16_t.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_bf16(const ApplyArgs &a, hipStream_t s) { return bp30_launch<bf16_t, bf16_t>(a, s); }
}  // namespace fem
