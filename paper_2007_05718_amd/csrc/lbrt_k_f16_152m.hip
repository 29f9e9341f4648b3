// Fused stream-collide kernel: f16_t storage, 152-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_152_moving() { return &launch_step<f16_t, 152, true>; }
}  // namespace lbrt
