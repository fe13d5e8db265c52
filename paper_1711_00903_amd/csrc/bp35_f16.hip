// BP3.5 kernels with f16_t storage.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f16(const ApplyArgs &a, hipStream_t s) { return bp35_launch<f16_t>(a, s); }
}  // namespace fem
