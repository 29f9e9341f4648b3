// Fused stream-collide kernel: float storage, 112-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_112_static() { return &launch_step<float, 112, false>; }
}  // namespace lbrt
