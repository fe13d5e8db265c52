// BP1.0 kernels with f16_t storage.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f16(const ApplyArgs &a, hipStream_t s) { return bp10_launch<f16_t>(a, s); }
}  // namespace fem
