// Fused stream-collide kernel: f16_t storage, 16-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_16_static() { return &launch_step<f16_t, 16, false>; }
}  // namespace lbrt
