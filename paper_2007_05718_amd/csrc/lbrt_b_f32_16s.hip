// Batched step kernel: float storage, 16-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchLauncher batch_f32_16_static() { return &launch_batch<float, 16, false>; }
}  // namespace lbrt
