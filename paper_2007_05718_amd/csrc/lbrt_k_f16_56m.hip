// Fused stream-collide kernel: f16_t storage, 56-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_56_moving() { return &launch_step<f16_t, 56, true>; }
}  // namespace lbrt
