// CG operator (stiffness + mass in one pass, FP64 fields) with geometric data stored as f16_t.
#include "cgop.hpp"

namespace fem {
hipError_t launch_cgop_f16g64(const CgopArgs &a, hipStream_t s) { return cgop_launch<f16_t>(a, s); }
}  // namespace fem
