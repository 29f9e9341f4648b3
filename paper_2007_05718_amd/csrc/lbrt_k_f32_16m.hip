// Fused stream-collide kernel: float storage, 16-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_16_moving() { return &launch_step<float, 16, true>; }
}  // namespace lbrt
