// BP3.0 kernels: geometric data stored as f16_t, fields as f16_t.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_f16(const ApplyArgs &a, hipStream_t s) { return bp30_launch<f16_t, f16_t>(a, s); }
}  // namespace fem
