// Step, init, batch and decode kernels for float64 storage and arithmetic.
#include "step_impl.h"

namespace rlbm {
RLBM_DEFINE_STORAGE_LAUNCHERS(double, double, f64)
}  // namespace rlbm
