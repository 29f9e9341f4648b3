// Fused stream-collide kernel: bf16_t storage, 112-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_112_static() { return &launch_step<bf16_t, 112, false>; }
}  // namespace lbrt
