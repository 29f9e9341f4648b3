// Fused stream-collide kernel: bf16_t storage, 32-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_32_static() { return &launch_step<bf16_t, 32, false>; }
}  // namespace lbrt
