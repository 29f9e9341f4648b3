// Fused stream-collide kernel: double storage, 152-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f64_152_static() { return &launch_step<double, 152, false>; }
}  // namespace lbrt
