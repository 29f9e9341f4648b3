// Fused stream-collide kernel: float storage, 160-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_160_static() { return &launch_step<float, 160, false>; }
}  // namespace lbrt
