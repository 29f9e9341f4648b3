// Fused stream-collide kernel: float storage, 56-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_56_moving() { return &launch_step<float, 56, true>; }
}  // namespace lbrt
