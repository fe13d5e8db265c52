// BP3.5 kernels: geometric data stored as bf16_t, fields as float.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_bf16g(const ApplyArgs &a, hipStream_t s) { return bp35_launch<bf16_t, float>(a, s); }
}  // namespace fem
