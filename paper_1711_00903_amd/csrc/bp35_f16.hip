// BP3.5 kernels: geometric data stored as f16_t, fields as f16_t.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f16(const ApplyArgs &a, hipStream_t s) { return bp35_launch<f16_t, f16_t>(a, s); }
}  // namespace fem
