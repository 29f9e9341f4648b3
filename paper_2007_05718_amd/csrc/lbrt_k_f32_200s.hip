// Fused stream-collide kernel: float storage, 200-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_200_static() { return &launch_step<float, 200, false>; }
}  // namespace lbrt
