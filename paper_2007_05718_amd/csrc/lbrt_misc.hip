// Small kernels around the fused step: moments of a stored state, storage
// conversion, deterministic reduction of the per-block diagnostics, fill.
#include "lbrt_step_kernel.h"

namespace lbrt {

// E = sum_i I_i, F = sum_i n_i I_i (eq. moments_discrete), summed in the
// table's processing order.
template <typename S>
__global__ void __launch_bounds__(kBlock)
moments_kernel(const S *__restrict__ I, const DirTab<typename StoreTraits<S>::T> *__restrict__ tab,
               int ndir, int64_t ncell, int64_t e_off, typename StoreTraits<S>::T *__restrict__ E,
               typename StoreTraits<S>::T *__restrict__ F) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  const int64_t cell = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  // FP64 sums (one thread per cell, memory-bound): in an optically thick
  // cell F is a small difference of terms of size E
  double e = 0.0, f0 = 0.0, f1 = 0.0, f2 = 0.0;
  for (int i = 0; i < ndir; ++i) {
    const DirTab<T> &d = tab[i];
    T v = Tr::ld(I + (int64_t)d.plane * ncell + cell);
    if (Tr::kReduced) v *= d.scale;
    if constexpr (Tr::kShifted)   // I_i = w_i E + s_i d_i
      v = fma(d.w, (T)reinterpret_cast<const float *>(
                       reinterpret_cast<const char *>(I) + e_off)[cell], v);
    const double vd = (double)v;
    e += vd;
    f0 = fma((double)d.n[0], vd, f0);
    f1 = fma((double)d.n[1], vd, f1);
    f2 = fma((double)d.n[2], vd, f2);
  }
  if (E) E[cell] = (T)e;
  if (F) {
    F[cell] = (T)f0;
    F[ncell + cell] = (T)f1;
    F[2 * ncell + cell] = (T)f2;
  }
}

template <typename S>
__device__ inline double load_phys(const void *p, int64_t i, double s) {
  using Tr = StoreTraits<S>;
  const double v = (double)Tr::ld(static_cast<const S *>(p) + i);
  return Tr::kReduced ? v * s : v;
}

template <typename S>
__device__ inline void store_phys(void *p, int64_t i, double v, double inv_s) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  Tr::st(static_cast<S *>(p) + i, Tr::kReduced ? (T)(v * inv_s) : (T)v);
}

// Conversion of a state between storage types, one element per thread (for
// an equilibrium-shifted source, I_i = w_i E + s_i d_i with the cell's E at
// byte e_off of the source; a shifted destination is written by
// shift_encode_kernel instead).
__global__ void __launch_bounds__(kBlock)
convert_kernel(const void *src, int src_storage, void *dst, int dst_storage,
               const double *__restrict__ scales, const double *__restrict__ weights, int ndir,
               int64_t ncell, int64_t e_off) {
  const int64_t total = ncell * ndir;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kBlock) {
    const double s = scales[i / ncell];
    double v;
    switch (src_storage) {
      case LBRT_FP32: v = load_phys<float>(src, i, s); break;
      case LBRT_FP64: v = load_phys<double>(src, i, s); break;
      case LBRT_BF16: v = load_phys<bf16_t>(src, i, s); break;
      case LBRT_FP16: v = load_phys<f16_t>(src, i, s); break;
      default: {
        const double E = (double)reinterpret_cast<const float *>(
            static_cast<const char *>(src) + e_off)[i % ncell];
        v = src_storage == LBRT_BF16_SHIFTED ? load_phys<bf16s_t>(src, i, s)
                                             : load_phys<f16s_t>(src, i, s);
        v = fma(weights[i / ncell], E, v);
        break;
      }
    }
    switch (dst_storage) {
      case LBRT_FP32: store_phys<float>(dst, i, v, 1.0 / s); break;
      case LBRT_FP64: store_phys<double>(dst, i, v, 1.0 / s); break;
      case LBRT_BF16: store_phys<bf16_t>(dst, i, v, 1.0 / s); break;
      default: store_phys<f16_t>(dst, i, v, 1.0 / s); break;
    }
  }
}

// An equilibrium-shifted state from any other: per cell (one thread), the
// FP64 sum of its populations in direction order, rounded to FP32, is the
// cell's E (stored at byte e_off of dst), and each population is stored as
// (I_i - w_i E) / s_i, rounded to nearest.
template <typename D>
__global__ void __launch_bounds__(kBlock)
shift_encode_kernel(const void *src, int src_storage, void *dst,
                    const double *__restrict__ scales, const double *__restrict__ weights,
                    int ndir, int64_t ncell, int64_t e_off) {
  const int64_t cell = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= ncell) return;
  auto phys = [&](int i) -> double {
    const int64_t k = (int64_t)i * ncell + cell;
    switch (src_storage) {
      case LBRT_FP32: return load_phys<float>(src, k, 1.0);
      case LBRT_FP64: return load_phys<double>(src, k, 1.0);
      case LBRT_BF16: return load_phys<bf16_t>(src, k, scales[i]);
      default: return load_phys<f16_t>(src, k, scales[i]);
    }
  };
  double e = 0.0;
  for (int i = 0; i < ndir; ++i) e += phys(i);
  const float E = (float)e;
  reinterpret_cast<float *>(static_cast<char *>(dst) + e_off)[cell] = E;
  for (int i = 0; i < ndir; ++i)
    store_phys<D>(dst, (int64_t)i * ncell + cell, phys(i) - weights[i] * (double)E,
                  1.0 / scales[i]);
}

// Fixed-order reduction of the step kernel's per-block partials into diag:
// block j of the grid reduces entry j.  Thread t sums blocks t, t + 256, ...
// in order, then a fixed tree over threads, so the result does not depend on
// timing.  Entries 1..7 (boundary fluxes) accumulate over steps; 0 and 8
// (sums of E and E*) hold the last step.
__global__ void __launch_bounds__(kBlock)
diag_reduce_kernel(const double *__restrict__ partials, int nblocks, double *__restrict__ diag,
                   int first_step) {
  __shared__ double red[kBlock];
  const int j = blockIdx.x;   // diag entry
  // partial columns: 0 sum E, 1 sum E*, 2..7 outflux per face, 8 influx
  const int col = j == 0 ? 0 : (j == 8 ? 1 : (j == 7 ? 8 : j + 1));
  double s = 0.0;
  // (unrolled so that several loads are in flight; the additions keep their
  // order)
#pragma unroll 8
  for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partials[(int64_t)b * kStepPartials + col];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (j == 0 || j == 8 || first_step) diag[j] = red[0];
    else diag[j] += red[0];
  }
}

// The ghost-plane table of a call, from its compact kernel-argument form.
__global__ void __launch_bounds__(kBlock)
inflow_table_kernel(const InflowCompact c, InflowArgs *__restrict__ out) {
  const int t = threadIdx.x;
  for (int k = t; k < LBRT_MAX_DIRS; k += kBlock)
    for (int a = 0; a < 3; ++a) {
      const int j = c.slot_plane[k][a];
      out->ghost[k][a] = j >= 0 ? c.ptr[j] : nullptr;
    }
  if (t < LBRT_MAX_INFLOW) {
    out->face[t] = c.face[t];
    out->dir[t] = c.dir[t];
    out->ptr[t] = c.ptr[t];
  }
  if (t == 0) out->n = c.n;
}

// Streaming copy, the bandwidth ceiling the step kernels are measured
// against: 16-byte loads, four in flight per lane, coalesced across the
// block, non-temporal 16-byte stores, grid-stride over the buffer.
constexpr int kCopyUnroll = 4;
typedef float f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kBlock)
stream_copy_kernel(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock * kCopyUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kBlock * kCopyUnroll + threadIdx.x; base < n;
       base += stride) {
    f32x4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kBlock;
      if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
  }
}

__global__ void fill_f64_kernel(double *p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_moments(int storage, const void *I, const void *tab, const KParams &p,
                          void *E, void *F, hipStream_t s) {
  const int nb = (int)((p.ncell + kBlock - 1) / kBlock);
  switch (storage) {
    case LBRT_FP32:
      hipLaunchKernelGGL(moments_kernel<float>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const float *>(I), static_cast<const DirTab<float> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<float *>(E), static_cast<float *>(F));
      break;
    case LBRT_FP64:
      hipLaunchKernelGGL(moments_kernel<double>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const double *>(I), static_cast<const DirTab<double> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<double *>(E), static_cast<double *>(F));
      break;
    case LBRT_BF16:
      hipLaunchKernelGGL(moments_kernel<bf16_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const bf16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<float *>(E), static_cast<float *>(F));
      break;
    case LBRT_FP16:
      hipLaunchKernelGGL(moments_kernel<f16_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const f16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<float *>(E),
                         static_cast<float *>(F));
      break;
    case LBRT_BF16_SHIFTED:
      hipLaunchKernelGGL(moments_kernel<bf16s_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const bf16s_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<float *>(E),
                         static_cast<float *>(F));
      break;
    default:
      hipLaunchKernelGGL(moments_kernel<f16s_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const f16s_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p.ndir, p.ncell, p.e_off, static_cast<float *>(E),
                         static_cast<float *>(F));
      break;
  }
  return hipGetLastError();
}

hipError_t launch_convert(const void *src, int src_storage, void *dst, int dst_storage,
                          const double *scales_dev, const double *weights_dev, int ndir,
                          int64_t ncell, int64_t e_off, hipStream_t s) {
  if (dst_storage == LBRT_BF16_SHIFTED || dst_storage == LBRT_FP16_SHIFTED) {
    const unsigned nb = (unsigned)((ncell + kBlock - 1) / kBlock);
    if (dst_storage == LBRT_BF16_SHIFTED)
      hipLaunchKernelGGL(shift_encode_kernel<bf16s_t>, dim3(nb), dim3(kBlock), 0, s, src,
                         src_storage, dst, scales_dev, weights_dev, ndir, ncell, e_off);
    else
      hipLaunchKernelGGL(shift_encode_kernel<f16s_t>, dim3(nb), dim3(kBlock), 0, s, src,
                         src_storage, dst, scales_dev, weights_dev, ndir, ncell, e_off);
    return hipGetLastError();
  }
  const int64_t total = ncell * ndir;
  int64_t nb = (total + kBlock - 1) / kBlock;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s, src, src_storage,
                     dst, dst_storage, scales_dev, weights_dev, ndir, ncell, e_off);
  return hipGetLastError();
}

hipError_t launch_diag_reduce(const double *partials, int nblocks, double *diag, int first_step,
                              hipStream_t s) {
  hipLaunchKernelGGL(diag_reduce_kernel, dim3(kDiag), dim3(kBlock), 0, s, partials, nblocks, diag,
                     first_step);
  return hipGetLastError();
}

// Blocks of the z-face flux kernel: the face cells in blocks of kBlock, times
// kZfaceGroups direction groups (each thread visits every kZfaceGroups-th
// direction, so that the grid has enough waves to hide the loads' latency).
int zface_blocks(const KParams &p) {
  if (p.periodic[2]) return 0;
  return (int)((2 * (int64_t)p.nx * p.ny + kBlock - 1) / kBlock) * kZfaceGroups;
}

hipError_t launch_zface(int storage, const void *I, const void *tab, const KParams &p,
                        const InflowArgs *inflow, double *partials, hipStream_t s) {
  const int nb = zface_blocks(p) / kZfaceGroups;
  if (nb == 0) return hipSuccess;
  const dim3 grid(nb, kZfaceGroups);
  switch (storage) {
    case LBRT_FP32:
      hipLaunchKernelGGL(zface_kernel<float>, grid, dim3(kBlock), 0, s,
                         static_cast<const float *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    case LBRT_FP64:
      hipLaunchKernelGGL(zface_kernel<double>, grid, dim3(kBlock), 0, s,
                         static_cast<const double *>(I),
                         static_cast<const DirTab<double> *>(tab), p, inflow, partials);
      break;
    case LBRT_BF16:
      hipLaunchKernelGGL(zface_kernel<bf16_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const bf16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    case LBRT_FP16:
      hipLaunchKernelGGL(zface_kernel<f16_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const f16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    case LBRT_BF16_SHIFTED:
      hipLaunchKernelGGL(zface_kernel<bf16s_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const bf16s_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    default:
      hipLaunchKernelGGL(zface_kernel<f16s_t>, grid, dim3(kBlock), 0, s,
                         static_cast<const f16s_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_inflow_table(const InflowCompact &c, InflowArgs *out, hipStream_t s) {
  hipLaunchKernelGGL(inflow_table_kernel, dim3(1), dim3(kBlock), 0, s, c, out);
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t s) {
  // eight blocks per CU on the 256 CUs, each lane looping over the rest
  int64_t nb = (n16 + (int64_t)kBlock * kCopyUnroll - 1) / ((int64_t)kBlock * kCopyUnroll);
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)nb), dim3(kBlock), 0, s,
                     static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n16);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace lbrt
