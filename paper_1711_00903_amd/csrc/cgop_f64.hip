// CG operator (stiffness + mass in one pass, FP64 fields) with geometric data stored as double.
#include "cgop.hpp"

namespace fem {
hipError_t launch_cgop_f64(const CgopArgs &a, hipStream_t s) { return cgop_launch<double>(a, s); }
}  // namespace fem
