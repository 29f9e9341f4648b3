// Fused stream-collide kernel: double storage, 56-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_56_moving() { return &launch_step<double, 56, true>; }
}  // namespace lbrt
