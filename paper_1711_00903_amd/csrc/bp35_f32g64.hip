// BP3.5 kernels: geometric data stored as float, fields as double.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f32g64(const ApplyArgs &a, hipStream_t s) { return bp35_launch<float, double>(a, s); }
}  // namespace fem
