// BP3.5 kernels: geometric data stored as double, fields as double.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f64(const ApplyArgs &a, hipStream_t s) { return bp35_launch<double, double>(a, s); }
}  // namespace fem
