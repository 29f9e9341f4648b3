// Fused stream-collide kernel: double storage, 112-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_112_moving() { return &launch_step<double, 112, true>; }
}  // namespace lbrt
