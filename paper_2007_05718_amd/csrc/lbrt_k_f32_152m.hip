// Fused stream-collide kernel: float storage, 152-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_152_moving() { return &launch_step<float, 152, true>; }
}  // namespace lbrt
