// Fused stream-collide kernel: float storage, 152-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_152_static() { return &launch_step<float, 152, false>; }
}  // namespace lbrt
