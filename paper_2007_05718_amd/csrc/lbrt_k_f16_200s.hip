// Fused stream-collide kernel: FP16 storage, 200-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_200_static() { return &launch_step<f16_t, 200, false>; }
}  // namespace lbrt
