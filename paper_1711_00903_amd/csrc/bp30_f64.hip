// BP3.0 kernels with double storage.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_f64(const ApplyArgs &a, hipStream_t s) { return bp30_launch<double>(a, s); }
}  // namespace fem
