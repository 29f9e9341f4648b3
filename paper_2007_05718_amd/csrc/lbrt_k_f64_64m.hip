// Fused stream-collide kernel: double storage, 64-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_64_moving() { return &launch_step<double, 64, true>; }
}  // namespace lbrt
