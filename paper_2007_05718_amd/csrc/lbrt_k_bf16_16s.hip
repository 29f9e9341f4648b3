// Fused stream-collide kernel: bf16_t storage, 16-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_16_static() { return &launch_step<bf16_t, 16, false>; }
}  // namespace lbrt
