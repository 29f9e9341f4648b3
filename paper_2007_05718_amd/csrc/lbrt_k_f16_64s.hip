// Fused stream-collide kernel: f16_t storage, 64-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_64_static() { return &launch_step<f16_t, 64, false>; }
}  // namespace lbrt
