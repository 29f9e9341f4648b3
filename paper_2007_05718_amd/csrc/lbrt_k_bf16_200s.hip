// Fused stream-collide kernel: BF16 storage, 200-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_bf16_200_static() { return &launch_step<bf16_t, 200, false>; }
}  // namespace lbrt
