// Fused stream-collide kernels for f16_t population storage, one per
// direction-count bucket.
#include "lbrt_step_kernel.h"

namespace lbrt {

StepLauncher step_launcher_f16(int bucket_index) {
  switch (bucket_index) {
    case 0: return &launch_step<f16_t, 16>;
    case 1: return &launch_step<f16_t, 32>;
    case 2: return &launch_step<f16_t, 50>;
    case 3: return &launch_step<f16_t, 64>;
    case 4: return &launch_step<f16_t, 110>;
    case 5: return &launch_step<f16_t, 128>;
    case 6: return &launch_step<f16_t, 146>;
    case 7: return &launch_step<f16_t, 160>;
    default: return nullptr;
  }
}

}  // namespace lbrt
