// BP3.5 kernels: geometric data stored as bf16_t, fields as bf16_t.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_bf16(const ApplyArgs &a, hipStream_t s) { return bp35_launch<bf16_t, bf16_t>(a, s); }
}  // namespace fem
