// Fused stream-collide kernel: float storage, 128-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f32_128_static() { return &launch_step<float, 128, false>; }
}  // namespace lbrt
