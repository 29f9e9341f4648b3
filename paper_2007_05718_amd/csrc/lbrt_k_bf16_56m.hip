// Fused stream-collide kernel: bf16_t storage, 56-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_56_moving() { return &launch_step<bf16_t, 56, true>; }
}  // namespace lbrt
