// Fused stream-collide kernel: double storage, 56-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_56_static() { return &launch_step<double, 56, false>; }
}  // namespace lbrt
