// Fused stream-collide kernel: float storage, 200-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_200_moving() { return &launch_step<float, 200, true>; }
}  // namespace lbrt
