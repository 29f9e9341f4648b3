// Fused stream-collide kernel: bf16_t storage, 56-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_56_static() { return &launch_step<bf16_t, 56, false>; }
}  // namespace lbrt
