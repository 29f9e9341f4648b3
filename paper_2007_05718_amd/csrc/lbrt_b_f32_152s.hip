// Batched persistent kernel: float storage, 152-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchKernel batch_f32_152_static() {
  return {&launch_batch<float, 152, false>, batch_blocks_per_cu<float, 152, false>()};
}
}  // namespace lbrt
