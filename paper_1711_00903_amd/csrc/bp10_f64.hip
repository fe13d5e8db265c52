// BP1.0 kernels: geometric data stored as double, fields as double.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f64(const ApplyArgs &a, hipStream_t s) { return bp10_launch<double, double>(a, s); }
}  // namespace fem
