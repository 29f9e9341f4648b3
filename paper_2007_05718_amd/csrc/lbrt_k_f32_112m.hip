// Fused stream-collide kernel: float storage, 112-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_112_moving() { return &launch_step<float, 112, true>; }
}  // namespace lbrt
