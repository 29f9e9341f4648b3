// Fused stream-collide kernel: f16_t storage, 152-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_152_static() { return &launch_step<f16_t, 152, false>; }
}  // namespace lbrt
