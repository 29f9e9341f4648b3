// Fused stream-collide kernels for float population storage, one per
// direction-count bucket.
#include "lbrt_step_kernel.h"

namespace lbrt {

StepLauncher step_launcher_f32(int bucket_index) {
  switch (bucket_index) {
    case 0: return &launch_step<float, 16>;
    case 1: return &launch_step<float, 32>;
    case 2: return &launch_step<float, 50>;
    case 3: return &launch_step<float, 64>;
    case 4: return &launch_step<float, 110>;
    case 5: return &launch_step<float, 128>;
    case 6: return &launch_step<float, 146>;
    case 7: return &launch_step<float, 160>;
    default: return nullptr;
  }
}

}  // namespace lbrt
