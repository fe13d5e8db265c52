// BP3.5 kernels with double storage.
#include "bp35.hpp"

namespace fem {
hipError_t launch_bp35_f64(const ApplyArgs &a, hipStream_t s) { return bp35_launch<double>(a, s); }
}  // namespace fem
