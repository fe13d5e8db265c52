// BP3.0 kernels with f16_t storage.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_f16(const ApplyArgs &a, hipStream_t s) { return bp30_launch<f16_t>(a, s); }
}  // namespace fem
