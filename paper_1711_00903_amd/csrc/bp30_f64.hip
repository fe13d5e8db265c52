// BP3.0 kernels: geometric data stored as double, fields as double.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_f64(const ApplyArgs &a, hipStream_t s) { return bp30_launch<double, double>(a, s); }
}  // namespace fem
