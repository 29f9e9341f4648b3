// Fused stream-collide kernel: bf16_t storage, 64-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_64_static() { return &launch_step<bf16_t, 64, false>; }
}  // namespace lbrt
