// Fused stream-collide kernel: bf16_t storage, 152-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_152_moving() { return &launch_step<bf16_t, 152, true>; }
}  // namespace lbrt
