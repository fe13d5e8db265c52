// BP1.0 kernels with double storage.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f64(const ApplyArgs &a, hipStream_t s) { return bp10_launch<double>(a, s); }
}  // namespace fem
