// Batched step kernel: float storage, 56-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchLauncher batch_f32_56_static() { return &launch_batch<float, 56, false>; }
}  // namespace lbrt
