// Fused stream-collide kernel: float storage, 32-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_32_static() { return &launch_step<float, 32, false>; }
}  // namespace lbrt
