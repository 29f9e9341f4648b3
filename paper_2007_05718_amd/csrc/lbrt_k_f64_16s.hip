// Fused stream-collide kernel: double storage, 16-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_16_static() { return &launch_step<double, 16, false>; }
}  // namespace lbrt
