// Batched form: many independent domains, each with its own grid, fields and
// step count, advanced together.
//
// Step s of the batch is ONE launch that covers every tile of every domain
// still running at step s (the domains are sorted by step count, so those
// form a prefix): block l of the launch takes the l-th (domain, tile) item of
// the step and runs the tile's z-march (the same device code as lbrt_step,
// main or general path).  Kernel boundaries order the steps, so there are no
// waits between blocks; a run is a fixed sequence of launches that a hipGraph
// captures and replays as one.
#pragma once

#include "lbrt_step_kernel.h"

namespace lbrt {

template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(64 * waves_for(NB)) batch_kernel(const BatchPlan bp, int s) {
  using T = typename StoreTraits<S>::T;
  // item within step s; XCD k takes the k-th contiguous run of items, so
  // neighbouring tiles of a domain share that XCD's L2
  const long long l = xcd_tile(blockIdx.x, gridDim.x);
  // domain: among the step's active prefix of the (sorted) domains
  int a = 0, b = bp.step_active[s];   // tile_prefix[a] <= l < tile_prefix[b]
  while (b - a > 1) {
    const int mid = (a + b) >> 1;
    if (bp.tile_prefix[mid] <= l) a = mid; else b = mid;
  }
  const BatchDomain &D = bp.dom[a];
  const int t = (int)(l - bp.tile_prefix[a]);
  KParams p = D.p;
  const bool last = s == D.nsteps - 1;
  if (last && (D.E || D.F)) p.flags |= KF_WRITE_EF;
  const S *Iin = static_cast<const S *>(D.I[s & 1]);
  S *Iout = static_cast<S *>(const_cast<void *>(D.I[(s + 1) & 1]));
  const DirTab<T> *tab = static_cast<const DirTab<T> *>(D.tab);
  const int4 w = D.tiles[t];
  T *E = last ? static_cast<T *>(D.E) : nullptr;
  T *F = last ? static_cast<T *>(D.F) : nullptr;
  if (w.w > 0)
    march<S, NB, MOVING, true>(Iin, Iout, D.ka, D.ks, D.eta, D.vel, tab, p, bp.noinflow, E, F,
                               nullptr, w.x, w.y, w.z, w.w);
  else
    march<S, NB, MOVING, false>(Iin, Iout, D.ka, D.ks, D.eta, D.vel, tab, p, bp.noinflow, E, F,
                                nullptr, w.x, w.y, w.z, -w.w);
}

// Launches the batch's steps [0, maxsteps): one launch per step.
template <typename S, int NB, bool MOVING>
hipError_t launch_batch(const BatchPlan &bp, const long long *step_items, hipStream_t st) {
  for (int s = 0; s < bp.maxsteps; ++s) {
    hipLaunchKernelGGL((batch_kernel<S, NB, MOVING>), dim3((unsigned)step_items[s]),
                       dim3(64 * waves_for(NB)), 0, st, bp, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lbrt
