// BP1.0 kernels: geometric data stored as bf16_t, fields as float.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_bf16g(const ApplyArgs &a, hipStream_t s) { return bp10_launch<bf16_t, float>(a, s); }
}  // namespace fem
