// Fused stream-collide kernel: double storage, 152-slot bucket, moving fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_152_moving() { return &launch_step<double, 152, true>; }
}  // namespace lbrt
