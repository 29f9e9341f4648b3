// Batched persistent kernel: float storage, 56-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchKernel batch_f32_56_static() {
  return {&launch_batch<float, 56, false>, batch_blocks_per_cu<float, 56, false>()};
}
}  // namespace lbrt
