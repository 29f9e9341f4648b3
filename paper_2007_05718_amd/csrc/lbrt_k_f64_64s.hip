// Fused stream-collide kernel: double storage, 64-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_64_static() { return &launch_step<double, 64, false>; }
}  // namespace lbrt
