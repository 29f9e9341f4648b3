// Batched form: many independent domains, each with its own grid, fields and
// step count, advanced by one persistent launch.
//
// The work is a queue of items (step s, domain, tile) in step-major order
// (all items of step s of every domain come before any item of step s + 1).
// Each block pops the next item with an atomic counter, waits until every
// tile of the previous step of that domain has completed (a per-domain
// counter), runs the tile's z-march (the same device code as lbrt_step,
// main or general path), and counts the tile done.  A block only ever waits
// for items with smaller queue indices, which were popped by blocks that are
// running, so the queue always drains; every wait is also bounded (a spin
// limit that raises an error flag and moves on), so every wave exits.
//
// Memory ordering across XCDs: a finished tile's stores are released at agent
// scope before its counter increment; the waiter's acquire at agent scope
// invalidates stale cache lines before the tile reads its inputs.
#pragma once

#include "lbrt_step_kernel.h"

namespace lbrt {

template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(kBlock) batch_kernel(const BatchPlan bp) {
  using T = typename StoreTraits<S>::T;
  __shared__ long long s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(bp.next, 1ull);
    __syncthreads();
    const long long g = s_item;
    if (g >= bp.total) break;
    // step: the last s with step_offset[s] <= g
    int lo = 0, hi = bp.maxsteps;   // step_offset[lo] <= g < step_offset[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (bp.step_offset[mid] <= g) lo = mid; else hi = mid;
    }
    const int s = lo;
    const long long l = g - bp.step_offset[s];
    // domain: among the step's active prefix of the (sorted) domains
    int a = 0, b = bp.step_active[s];   // tile_prefix[a] <= l < tile_prefix[b]
    while (b - a > 1) {
      const int mid = (a + b) >> 1;
      if (bp.tile_prefix[mid] <= l) a = mid; else b = mid;
    }
    const int k = a;
    const BatchDomain &D = bp.dom[k];
    const int t = (int)(l - bp.tile_prefix[k]);
    if (s > 0 && threadIdx.x == 0) {
      // every tile of step s - 1 of this domain is done
      const unsigned long long need = (unsigned long long)s * (unsigned long long)D.ntiles;
      unsigned it = 0;
      while (__hip_atomic_load(&bp.done[k], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
        __builtin_amdgcn_s_sleep(4);
        if (++it >= kBatchSpinLimit) {
          atomicOr(bp.error, 1u);
          break;
        }
      }
    }
    __syncthreads();
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
      march<S, NB, MOVING, false>(Iin, Iout, D.ka, D.ks, D.eta, D.vel, tab, p, bp.noinflow, E,
                                  F, nullptr, w.x, w.y, w.z, -w.w);
    // every wave's stores reach memory before the tile is counted
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(&bp.done[k], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <typename S, int NB, bool MOVING>
hipError_t launch_batch(const BatchPlan &bp, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((batch_kernel<S, NB, MOVING>), dim3(nblocks), dim3(kBlock), 0, s, bp);
  return hipGetLastError();
}

template <typename S, int NB, bool MOVING>
int batch_blocks_per_cu() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<S, NB, MOVING>, kBlock, 0) !=
      hipSuccess)
    return 1;
  return n > 0 ? n : 1;
}

}  // namespace lbrt
