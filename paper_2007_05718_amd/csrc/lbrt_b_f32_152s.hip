// Batched step kernel: float storage, 152-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchLauncher batch_f32_152_static() { return &launch_batch<float, 152, false>; }
}  // namespace lbrt
