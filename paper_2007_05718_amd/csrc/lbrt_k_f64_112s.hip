// Fused stream-collide kernel: double storage, 112-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_112_static() { return &launch_step<double, 112, false>; }
}  // namespace lbrt
