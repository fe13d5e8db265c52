// BP3.0 kernels: geometric data stored as float, fields as float.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_f32(const ApplyArgs &a, hipStream_t s) { return bp30_launch<float, float>(a, s); }
}  // namespace fem
