// Fused stream-collide kernel: float storage, 56-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_56_static() { return &launch_step<float, 56, false>; }
}  // namespace lbrt
