// Fused stream-collide kernel: float storage, 64-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_64_static() { return &launch_step<float, 64, false>; }
}  // namespace lbrt
