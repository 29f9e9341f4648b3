// Fused stream-collide kernel: double storage, 32-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_32_static() { return &launch_step<double, 32, false>; }
}  // namespace lbrt
