// Table of the compiled (storage, bucket, fluid) kernel combinations.
#include "lbrt_internal.h"

namespace lbrt {

StepLauncher launcher_f32_16_static();
StepLauncher launcher_f32_16_moving();
StepLauncher launcher_f32_32_static();
StepLauncher launcher_f32_32_moving();
StepLauncher launcher_f32_56_static();
StepLauncher launcher_f32_56_moving();
StepLauncher launcher_f32_112_static();
StepLauncher launcher_f32_112_moving();
StepLauncher launcher_f32_152_static();
StepLauncher launcher_f32_152_moving();
StepLauncher launcher_f64_16_static();
StepLauncher launcher_f64_16_moving();
StepLauncher launcher_f64_32_static();
StepLauncher launcher_f64_32_moving();
StepLauncher launcher_f64_56_static();
StepLauncher launcher_f64_56_moving();
StepLauncher launcher_bf16_16_static();
StepLauncher launcher_bf16_32_static();
StepLauncher launcher_bf16_56_static();
StepLauncher launcher_bf16_56_moving();
StepLauncher launcher_bf16_112_static();
StepLauncher launcher_bf16_152_static();
StepLauncher launcher_bf16_152_moving();
StepLauncher launcher_f16_16_static();
StepLauncher launcher_f16_32_static();
StepLauncher launcher_f16_56_static();
StepLauncher launcher_f16_56_moving();
StepLauncher launcher_f16_112_static();
StepLauncher launcher_f16_152_static();
StepLauncher launcher_f16_152_moving();
StepLauncher launcher_bf16s_56_static();
StepLauncher launcher_bf16s_112_static();
StepLauncher launcher_f16s_56_static();
StepLauncher launcher_f16s_112_static();
StepLauncher launcher_f32_200_static();
StepLauncher launcher_f32_200_moving();
StepLauncher launcher_bf16_200_static();
StepLauncher launcher_f16_200_static();
StepLauncher launcher_f64_112_static();
StepLauncher launcher_f64_112_moving();
StepLauncher launcher_f64_152_static();
StepLauncher launcher_f64_152_moving();

StepLauncher step_launcher(int storage, int bucket_index, bool moving) {
  if (bucket_index < 0 || bucket_index >= kNumBuckets) return nullptr;
  const int nb = kBuckets[bucket_index];
  if (storage == LBRT_FP32 && nb == 16 && moving == false) return launcher_f32_16_static();
  if (storage == LBRT_FP32 && nb == 16 && moving == true) return launcher_f32_16_moving();
  if (storage == LBRT_FP32 && nb == 32 && moving == false) return launcher_f32_32_static();
  if (storage == LBRT_FP32 && nb == 32 && moving == true) return launcher_f32_32_moving();
  if (storage == LBRT_FP32 && nb == 56 && moving == false) return launcher_f32_56_static();
  if (storage == LBRT_FP32 && nb == 56 && moving == true) return launcher_f32_56_moving();
  if (storage == LBRT_FP32 && nb == 112 && moving == false) return launcher_f32_112_static();
  if (storage == LBRT_FP32 && nb == 112 && moving == true) return launcher_f32_112_moving();
  if (storage == LBRT_FP32 && nb == 152 && moving == false) return launcher_f32_152_static();
  if (storage == LBRT_FP32 && nb == 152 && moving == true) return launcher_f32_152_moving();
  if (storage == LBRT_FP64 && nb == 16 && moving == false) return launcher_f64_16_static();
  if (storage == LBRT_FP64 && nb == 16 && moving == true) return launcher_f64_16_moving();
  if (storage == LBRT_FP64 && nb == 32 && moving == false) return launcher_f64_32_static();
  if (storage == LBRT_FP64 && nb == 32 && moving == true) return launcher_f64_32_moving();
  if (storage == LBRT_FP64 && nb == 56 && moving == false) return launcher_f64_56_static();
  if (storage == LBRT_FP64 && nb == 56 && moving == true) return launcher_f64_56_moving();
  if (storage == LBRT_BF16 && nb == 16 && moving == false) return launcher_bf16_16_static();
  if (storage == LBRT_BF16 && nb == 32 && moving == false) return launcher_bf16_32_static();
  if (storage == LBRT_BF16 && nb == 56 && moving == false) return launcher_bf16_56_static();
  if (storage == LBRT_BF16 && nb == 56 && moving == true) return launcher_bf16_56_moving();
  if (storage == LBRT_BF16 && nb == 112 && moving == false) return launcher_bf16_112_static();
  if (storage == LBRT_BF16 && nb == 152 && moving == false) return launcher_bf16_152_static();
  if (storage == LBRT_BF16 && nb == 152 && moving == true) return launcher_bf16_152_moving();
  if (storage == LBRT_FP16 && nb == 16 && moving == false) return launcher_f16_16_static();
  if (storage == LBRT_FP16 && nb == 32 && moving == false) return launcher_f16_32_static();
  if (storage == LBRT_FP16 && nb == 56 && moving == false) return launcher_f16_56_static();
  if (storage == LBRT_FP16 && nb == 56 && moving == true) return launcher_f16_56_moving();
  if (storage == LBRT_FP16 && nb == 112 && moving == false) return launcher_f16_112_static();
  if (storage == LBRT_FP16 && nb == 152 && moving == false) return launcher_f16_152_static();
  if (storage == LBRT_FP16 && nb == 152 && moving == true) return launcher_f16_152_moving();
  if (storage == LBRT_BF16_SHIFTED && nb == 56 && moving == false) return launcher_bf16s_56_static();
  if (storage == LBRT_BF16_SHIFTED && nb == 112 && moving == false) return launcher_bf16s_112_static();
  if (storage == LBRT_FP16_SHIFTED && nb == 56 && moving == false) return launcher_f16s_56_static();
  if (storage == LBRT_FP16_SHIFTED && nb == 112 && moving == false) return launcher_f16s_112_static();
  if (storage == LBRT_FP32 && nb == 200 && moving == false) return launcher_f32_200_static();
  if (storage == LBRT_FP32 && nb == 200 && moving == true) return launcher_f32_200_moving();
  if (storage == LBRT_BF16 && nb == 200 && moving == false) return launcher_bf16_200_static();
  if (storage == LBRT_FP16 && nb == 200 && moving == false) return launcher_f16_200_static();
  if (storage == LBRT_FP64 && nb == 112 && moving == false) return launcher_f64_112_static();
  if (storage == LBRT_FP64 && nb == 112 && moving == true) return launcher_f64_112_moving();
  if (storage == LBRT_FP64 && nb == 152 && moving == false) return launcher_f64_152_static();
  if (storage == LBRT_FP64 && nb == 152 && moving == true) return launcher_f64_152_moving();
  return nullptr;
}

bool pair_available(int storage, int nb, bool moving) {
  return !moving &&
         (storage == LBRT_BF16 || storage == LBRT_FP16 || storage == LBRT_BF16_SHIFTED ||
          storage == LBRT_FP16_SHIFTED) &&
         (nb == 56 || nb == 112);
}

BatchLauncher batch_f32_16_static();
BatchLauncher batch_f32_32_static();
BatchLauncher batch_f32_56_static();
BatchLauncher batch_f32_112_static();
BatchLauncher batch_f32_152_static();

// Batched kernels exist for FP32 storage and a static fluid.
BatchLauncher batch_launcher(int storage, int bucket_index, bool moving) {
  if (bucket_index < 0 || bucket_index >= kNumBuckets) return nullptr;
  const int nb = kBuckets[bucket_index];
  if (storage == LBRT_FP32 && nb == 16 && !moving) return batch_f32_16_static();
  if (storage == LBRT_FP32 && nb == 32 && !moving) return batch_f32_32_static();
  if (storage == LBRT_FP32 && nb == 56 && !moving) return batch_f32_56_static();
  if (storage == LBRT_FP32 && nb == 112 && !moving) return batch_f32_112_static();
  if (storage == LBRT_FP32 && nb == 152 && !moving) return batch_f32_152_static();
  return nullptr;
}

}  // namespace lbrt
