// Fused stream-collide kernel: FP16 equilibrium-shifted storage, 112-slot
// bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16s_112_static() { return &launch_step<f16s_t, 112, false>; }
}  // namespace lbrt
