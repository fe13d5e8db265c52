// BP1.0 kernels with float storage.
#include "bp10.hpp"

namespace fem {
hipError_t launch_bp10_f32(const ApplyArgs &a, hipStream_t s) { return bp10_launch<float>(a, s); }
}  // namespace fem
