// Batched form: many independent domains, each with its own grid, fields and
// step count, advanced together.
//
// Step s of the batch is two launches (general-path tiles, then main-path
// tiles) that cover every tile of every domain still running at step s (the
// domains are sorted by step count, so those form a prefix): each block takes
// one (domain, tile) item and runs the tile's z-march (the same device code as
// lbrt_step).  Kernel boundaries order the steps, so there are no waits
// between blocks; a run is a fixed sequence of launches that a hipGraph
// captures and replays as one.
#pragma once

#include "lbrt_step_kernel.h"

namespace lbrt {

// One item of step s: block l of the launch takes the l-th (domain, tile)
// item of the step's main-path (MAIN) or general-path tiles.  The main and
// general paths are separate kernels so that each gets its own register
// budget (the general path's per-tap checks need more).
template <typename S, int NB, bool MOVING, bool MAIN>
__device__ __forceinline__ void batch_item(const BatchPlan &bp, const char *__restrict__ tabs,
                                           char *gbase, int s) {
  using T = typename StoreTraits<S>::T;
  const long long *prefix = MAIN ? bp.main_prefix : bp.gen_prefix;
  // item within step s; XCD k takes the k-th contiguous run of items, so
  // neighbouring tiles of a domain share that XCD's L2
  const long long l = xcd_tile(blockIdx.x, gridDim.x);
  // domain: among the step's active prefix of the (sorted) domains
  int a = 0, b = bp.step_active[s];   // prefix[a] <= l < prefix[b]
  while (b - a > 1) {
    const int mid = (a + b) >> 1;
    if (prefix[mid] <= l) a = mid; else b = mid;
  }
  // the search is the same in every lane: say so, so that the domain's
  // fields, pointers and direction table are read with scalar loads
  a = __builtin_amdgcn_readfirstlane(a);
  const BatchDomain &D = bp.dom[a];
  const int t = __builtin_amdgcn_readfirstlane((int)(l - prefix[a]));
  KParams p = D.p;
  const bool last = s == D.nsteps - 1;
  if (last && (D.E != kNoBuffer || D.F != kNoBuffer)) p.flags |= KF_WRITE_EF;
  // offsets and the tile are the same in every lane: keep them in scalar
  // registers, so that table reads are scalar loads and buffer bases uniform
  auto u64 = [](int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  auto buf = [&](int64_t off) -> char * {
    off = u64(off);
    return off == kNoBuffer ? nullptr : gbase + off;
  };
  const S *Iin = reinterpret_cast<const S *>(gbase + u64(D.I[s & 1]));
  S *Iout = reinterpret_cast<S *>(gbase + u64(D.I[(s + 1) & 1]));
  const DirTab<T> *tab = reinterpret_cast<const DirTab<T> *>(tabs + u64(D.tab));
  // the tile: main tiles are (x0, y0, zb, ze) of the context's tile shape,
  // general ones carry their own shape and bounds
  int x0, y0, zb, ze, txlog = p.txlog, xe = p.nx, ye = p.ny;
  if constexpr (MAIN) {
    const int4 w = D.tiles[t];
    x0 = w.x, y0 = w.y, zb = w.z, ze = w.w;
  } else {
    const GenTile g = D.gtiles[t];
    x0 = g.x0, y0 = g.y0, zb = g.zb, ze = g.ze, txlog = g.txlog, xe = g.xe, ye = g.ye;
  }
  x0 = __builtin_amdgcn_readfirstlane(x0);
  y0 = __builtin_amdgcn_readfirstlane(y0);
  zb = __builtin_amdgcn_readfirstlane(zb);
  ze = __builtin_amdgcn_readfirstlane(ze);
  txlog = __builtin_amdgcn_readfirstlane(txlog);
  xe = __builtin_amdgcn_readfirstlane(xe);
  ye = __builtin_amdgcn_readfirstlane(ye);
  T *E = last ? reinterpret_cast<T *>(buf(D.E)) : nullptr;
  T *F = last ? reinterpret_cast<T *>(buf(D.F)) : nullptr;
  march<S, NB, MOVING, MAIN>(Iin, Iout, reinterpret_cast<const float *>(gbase + u64(D.ka)),
                             reinterpret_cast<const float *>(gbase + u64(D.ks)),
                             reinterpret_cast<const float *>(gbase + u64(D.eta)),
                             reinterpret_cast<const float *>(buf(D.vel)), tab, p, bp.noinflow,
                             E, F, nullptr, x0, y0, zb, ze, txlog, xe, ye);
}

template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(64 * waves_for(NB), waves_per_simd<S>(NB))
batch_kernel_main(const BatchPlan bp, const char *__restrict__ tabs, char *gbase, int s) {
  batch_item<S, NB, MOVING, true>(bp, tabs, gbase, s);
}

template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(64 * waves_for(NB))
batch_kernel_general(const BatchPlan bp, const char *__restrict__ tabs, char *gbase, int s) {
  batch_item<S, NB, MOVING, false>(bp, tabs, gbase, s);
}

// Launches the batch's steps [0, maxsteps): per step the general-path tiles,
// then the main-path tiles (both read step s's buffer and write the other).
template <typename S, int NB, bool MOVING>
hipError_t launch_batch(const BatchPlan &bp, const long long *step_main,
                        const long long *step_gen, hipStream_t st) {
  for (int s = 0; s < bp.maxsteps; ++s) {
    if (step_gen[s] > 0)
      hipLaunchKernelGGL((batch_kernel_general<S, NB, MOVING>), dim3((unsigned)step_gen[s]),
                         dim3(64 * waves_for(NB)), 0, st, bp, bp.tabs, bp.gbase, s);
    if (step_main[s] > 0)
      hipLaunchKernelGGL((batch_kernel_main<S, NB, MOVING>), dim3((unsigned)step_main[s]),
                         dim3(64 * waves_for(NB)), 0, st, bp, bp.tabs, bp.gbase, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lbrt
