// BP3.5 kernels: geometric data stored as float, fields as float.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f32(const ApplyArgs &a, hipStream_t s) { return bp35_launch<float, float>(a, s); }
}  // namespace fem
