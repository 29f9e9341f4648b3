// Fused stream-collide kernel: bf16_t storage, 152-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_152_static() { return &launch_step<bf16_t, 152, false>; }
}  // namespace lbrt
