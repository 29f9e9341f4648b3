// Batched persistent kernel: float storage, 32-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchKernel batch_f32_32_static() {
  return {&launch_batch<float, 32, false>, batch_blocks_per_cu<float, 32, false>()};
}
}  // namespace lbrt
