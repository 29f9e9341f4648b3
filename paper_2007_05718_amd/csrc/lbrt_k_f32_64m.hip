// Fused stream-collide kernel: float storage, 64-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_64_moving() { return &launch_step<float, 64, true>; }
}  // namespace lbrt
