// Fused stream-collide kernel: double storage, 32-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_32_moving() { return &launch_step<double, 32, true>; }
}  // namespace lbrt
