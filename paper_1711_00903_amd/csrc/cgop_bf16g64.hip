// CG operator (stiffness + mass in one pass, FP64 fields) with geometric data stored as bf16_t.
#include "cgop.hpp"

namespace fem {
hipError_t launch_cgop_bf16g64(const CgopArgs &a, hipStream_t s) { return cgop_launch<bf16_t>(a, s); }
}  // namespace fem
