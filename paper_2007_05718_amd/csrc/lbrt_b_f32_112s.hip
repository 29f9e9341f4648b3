// Batched step kernel: float storage, 112-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchLauncher batch_f32_112_static() { return &launch_batch<float, 112, false>; }
}  // namespace lbrt
