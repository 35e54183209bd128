// Step, init, batch and decode kernels for float32 storage and arithmetic.
#include "step_impl.h"

namespace rlbm {
RLBM_DEFINE_STORAGE_LAUNCHERS(float, float, f32)
}  // namespace rlbm
