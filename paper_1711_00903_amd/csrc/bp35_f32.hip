// BP3.5 kernels with float storage.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f32(const ApplyArgs &a, hipStream_t s) { return bp35_launch<float>(a, s); }
}  // namespace fem
