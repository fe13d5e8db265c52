// BP1.0 kernels: geometric data stored as float, fields as double.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f32g64(const ApplyArgs &a, hipStream_t s) { return bp10_launch<float, double>(a, s); }
}  // namespace fem
