// Fused stream-collide kernel: double storage, 16-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_16_moving() { return &launch_step<double, 16, true>; }
}  // namespace lbrt
