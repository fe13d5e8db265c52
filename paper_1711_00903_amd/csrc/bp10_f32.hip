// BP1.0 kernels: geometric data stored as float, fields as float.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f32(const ApplyArgs &a, hipStream_t s) { return bp10_launch<float, float>(a, s); }
}  // namespace fem
