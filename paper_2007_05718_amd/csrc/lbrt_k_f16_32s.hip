// Fused stream-collide kernel: f16_t storage, 32-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_32_static() { return &launch_step<f16_t, 32, false>; }
}  // namespace lbrt
