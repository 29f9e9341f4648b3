// Boundary energy fluxes of one streaming step, computed from the state that
// enters the step.  Only the six face layers are touched.
//
// Outflux: a population on the downstream face layer of axis a sends the
// fraction dt |n^a| / dx of itself out through that face (eq. interp); when
// it leaves along several axes at once the part that is outside in x is
// booked on the x face, the rest that is outside in y on the y face, the
// rest on the z face.  Influx: the taps of face-layer cells that read an
// inflow ghost value (a point outside along that face's axis only).
#include "lbrt_step_kernel.h"

namespace lbrt {

namespace {

constexpr int kFaceGrid = 512;

template <typename S>
__global__ void __launch_bounds__(kBlock)
face_flux_kernel(const S *__restrict__ I,
                 const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams p,
                 const InflowArgs *__restrict__ inflow, double *__restrict__ partials) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int n3[3] = {nx, ny, nz};
  const int64_t fx = (int64_t)ny * nz, fy = (int64_t)nx * nz, fz = (int64_t)nx * ny;
  const int64_t total = 2 * (fx + fy + fz);
  double acc[kFacePartials];
#pragma unroll
  for (int j = 0; j < kFacePartials; ++j) acc[j] = 0.0;

  for (int64_t w = (int64_t)blockIdx.x * kBlock + threadIdx.x; w < total;
       w += (int64_t)gridDim.x * kBlock) {
    // decode (face, cell)
    int f;
    int64_t r = w;
    if (r < 2 * fx) { f = (int)(r / fx); r -= f * fx; }
    else if ((r -= 2 * fx) < 2 * fy) { f = 2 + (int)(r / fy); r -= (f - 2) * fy; }
    else { r -= 2 * fy; f = 4 + (int)(r / fz); r -= (f - 4) * fz; }
    const int a = f >> 1, hi = f & 1;
    int c[3];
    if (a == 0) { c[1] = (int)(r % ny); c[2] = (int)(r / ny); c[0] = hi ? nx - 1 : 0; }
    else if (a == 1) { c[0] = (int)(r % nx); c[2] = (int)(r / nx); c[1] = hi ? ny - 1 : 0; }
    else { c[0] = (int)(r % nx); c[1] = (int)(r / nx); c[2] = hi ? nz - 1 : 0; }
    if (p.periodic[a]) continue;
    const int64_t cell = ((int64_t)c[2] * ny + c[1]) * nx + c[0];
    bool has_ghosts = false;
    for (int j = 0; j < inflow->n; ++j) has_ghosts |= inflow->face[j] == f;
    for (int k = 0; k < p.ndir; ++k) {
      const DirTab<T> &d = tab[k];
      const int sa = d.s[a];
      const bool leaving = hi ? sa > 0 : sa < 0;
      if (leaving) {
        T stay = T(1);
        for (int b = 0; b < a; ++b) {
          const int sb = d.s[b];
          if (sb != 0 && !p.periodic[b]) {
            const bool at = sb > 0 ? c[b] == n3[b] - 1 : c[b] == 0;
            if (at) stay *= T(1) - d.delta[b];
          }
        }
        T v = Tr::ld(I + (int64_t)d.plane * p.ncell + cell);
        if (Tr::kReduced) v *= d.scale;
        acc[f] += (double)(stay * d.delta[a] * v);
      }
      // ghost values that enter through face f
      const bool entering = hi ? sa < 0 : sa > 0;
      if (entering && has_ghosts) {
        const float *g = nullptr;
        for (int j = 0; j < inflow->n; ++j)
          if (inflow->face[j] == f && inflow->dir[j] == d.plane) g = inflow->ptr[j];
        if (g != nullptr) {
          // taps shifted along a; the other two coordinates must stay in the box
          const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;
          T in = T(0);
          for (int b = 0; b < 8; ++b) {
            if (((b >> a) & 1) == 0) continue;
            int u = c[o1] - ((b >> o1) & 1) * d.s[o1];
            int v = c[o2] - ((b >> o2) & 1) * d.s[o2];
            if (p.periodic[o1]) u = u < 0 ? u + n3[o1] : (u >= n3[o1] ? u - n3[o1] : u);
            if (p.periodic[o2]) v = v < 0 ? v + n3[o2] : (v >= n3[o2] ? v - n3[o2] : v);
            if ((unsigned)u >= (unsigned)n3[o1] || (unsigned)v >= (unsigned)n3[o2]) continue;
            // plane layouts: x faces [z][y], y faces [z][x], z faces [y][x]
            const int64_t gi = (int64_t)v * n3[o1] + u;
            in += d.tw[b] * (T)g[gi];
          }
          acc[6] += (double)in;
        }
      }
    }
  }
  block_sums<kFacePartials>(acc, partials + (int64_t)blockIdx.x * kFacePartials);
}

}  // namespace

int face_flux_blocks(const KParams &p) {
  const int64_t total = 2 * ((int64_t)p.ny * p.nz + (int64_t)p.nx * p.nz + (int64_t)p.nx * p.ny);
  const int64_t need = (total + kBlock - 1) / kBlock;
  return (int)(need < kFaceGrid ? need : kFaceGrid);
}

hipError_t launch_face_flux(int storage, const void *I, const void *tab, const KParams &p,
                            const InflowArgs *inflow, double *partials, int *nblocks,
                            hipStream_t s) {
  const int nb = face_flux_blocks(p);
  *nblocks = nb;
  switch (storage) {
    case LBRT_FP32:
      hipLaunchKernelGGL(face_flux_kernel<float>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const float *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    case LBRT_FP64:
      hipLaunchKernelGGL(face_flux_kernel<double>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const double *>(I),
                         static_cast<const DirTab<double> *>(tab), p, inflow, partials);
      break;
    case LBRT_BF16:
      hipLaunchKernelGGL(face_flux_kernel<bf16_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const bf16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
    default:
      hipLaunchKernelGGL(face_flux_kernel<f16_t>, dim3(nb), dim3(kBlock), 0, s,
                         static_cast<const f16_t *>(I), static_cast<const DirTab<float> *>(tab),
                         p, inflow, partials);
      break;
  }
  return hipGetLastError();
}

}  // namespace lbrt
