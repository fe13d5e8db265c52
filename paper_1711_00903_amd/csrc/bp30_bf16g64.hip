// BP3.0 kernels: geometric data stored as bf16_t, fields as double.
#include "bp30.hpp"

namespace fem {
hipError_t launch_bp30_bf16g64(const ApplyArgs &a, hipStream_t s) { return bp30_launch<bf16_t, double>(a, s); }
}  // namespace fem
