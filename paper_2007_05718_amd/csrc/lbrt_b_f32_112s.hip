// Batched persistent kernel: float storage, 112-slot bucket, static fluid.
#include "lbrt_batch_kernel.h"

namespace lbrt {
BatchKernel batch_f32_112_static() {
  return {&launch_batch<float, 112, false>, batch_blocks_per_cu<float, 112, false>()};
}
}  // namespace lbrt
