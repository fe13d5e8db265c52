// CG operator (stiffness + mass in one pass, FP64 fields) with geometric data stored as float.
#include "cgop.hpp"

namespace fem {
hipError_t launch_cgop_f32g64(const CgopArgs &a, hipStream_t s) { return cgop_launch<float>(a, s); }
}  // namespace fem
