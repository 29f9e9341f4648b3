// Fused stream-collide kernel: float storage, 32-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_32_moving() { return &launch_step<float, 32, true>; }
}  // namespace lbrt
