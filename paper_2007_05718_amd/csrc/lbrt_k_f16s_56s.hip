// Fused stream-collide kernel: FP16 equilibrium-shifted storage, 56-slot
// bucket, static fluid.
#include "lbrt_step_kernel.h"

namespace lbrt {
StepLauncher launcher_f16s_56_static() { return &launch_step<f16s_t, 56, false>; }
}  // namespace lbrt
