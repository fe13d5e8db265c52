// BP1.0 kernels: geometric data stored as bf16_t, fields as bf16_t.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_bf16(const ApplyArgs &a, hipStream_t s) { return bp10_launch<bf16_t, bf16_t>(a, s); }
}  // namespace fem
