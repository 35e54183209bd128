// Step, init, batch and decode kernels for float16 deviation storage, float32 arithmetic.
#include "step_impl.h"

namespace rlbm {
RLBM_DEFINE_STORAGE_LAUNCHERS(_Float16, float, f16)
}  // namespace rlbm
