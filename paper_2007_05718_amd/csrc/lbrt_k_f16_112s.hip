// Fused stream-collide kernel: f16_t storage, 112-slot bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16_112_static() { return &launch_step<f16_t, 112, false>; }
}  // namespace lbrt
