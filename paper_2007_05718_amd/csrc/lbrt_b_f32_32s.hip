// Batched step kernel: float storage, 32-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchLauncher batch_f32_32_static() { return &launch_batch<float, 32, false>; }
}  // namespace lbrt
