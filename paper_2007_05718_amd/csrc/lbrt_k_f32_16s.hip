// Fused stream-collide kernel: float storage, 16-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_16_static() { return &launch_step<float, 16, false>; }
}  // namespace lbrt
