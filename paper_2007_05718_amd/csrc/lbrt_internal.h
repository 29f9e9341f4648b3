// Internal types shared by the host dispatcher and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbrt.h"

namespace lbrt {

// 16-bit storage wrappers (bit patterns; conversions live in the kernels).
struct bf16_t { uint16_t u; };
struct f16_t { uint16_t u; };

// Per-direction constants, in processing order (antipodal pairs adjacent
// when the rule is centrally symmetric).  Zero-weight taps of degenerate
// directions (a zero component) are collapsed onto the tap with the same
// other shifts, so every tap of an in-box cell is an in-box address.
template <typename T>
struct DirTab {
  T w;            // quadrature weight
  T n[3];         // unit direction
  T tw[8];        // trilinear tap weights, tap b = bx | by << 1 | bz << 2
  T delta[3];     // dt |n^a| / dx, the fraction pulled from the upwind cell
  T scale;        // storage scale s_i (1 for FP32/FP64)
  T inv_scale;    // 1 / s_i
  int32_t s[3];   // effective shift signs: sgn(n^a), 0 where n^a == 0
  int32_t off[8]; // element offset of tap b: -(bx sx + by sy nx + bz sz nx ny)
  int32_t plane;  // storage plane (direction index in the caller's order)
  int32_t pad;
};

struct InflowArgs {
  int32_t n;
  int32_t face[LBRT_MAX_INFLOW];
  int32_t dir[LBRT_MAX_INFLOW];      // storage plane index
  const float *ptr[LBRT_MAX_INFLOW];
};

enum : uint32_t {
  KF_PAIRED = 1u << 0,   // directions come in antipodal pairs (2k, 2k+1)
  KF_MOVING = 1u << 1,   // mixed-frame collision (App. B)
  KF_DIAG = 1u << 2,     // accumulate diagnostics into per-block partials
  KF_WRITE_EF = 1u << 3, // write E, F of the new state
  KF_LAMZERO = 1u << 4,  // lambda == 0 (anisotropic term skipped)
};

struct KParams {
  int32_t nx, ny, nz;
  int32_t ndir;
  int64_t ncell;
  int32_t tx, ty, tz;          // tile shape (== block shape)
  int32_t ntx, nty, ntz;       // tiles per axis
  int32_t ntiles;
  int32_t periodic[3];         // per axis x, y, z
  int32_t inflow_face[6];      // face is an inflow face
  int32_t mode;                // lbrt_collision
  int32_t lambda_iters;
  uint32_t flags;
  double dt;
  double lam;
};

constexpr int kBlock = 256;
constexpr int kDiag = LBRT_DIAG_LEN;

// Direction-count buckets with a compiled kernel.  Rules whose size is
// not a bucket run in the next larger bucket, padded with null directions.
constexpr int kBuckets[] = {16, 32, 50, 64, 110, 128, 146, 160};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);

// Launchers, one per (storage, bucket), defined in lbrt_step_*.hip.
using StepLauncher = hipError_t (*)(const void *Iin, void *Iout, const float *ka,
                                    const float *ks, const float *eta, const float *vel,
                                    const void *tab, const KParams &p,
                                    const InflowArgs &inflow, void *E, void *F,
                                    double *partials, hipStream_t s);

StepLauncher step_launcher(int storage, int bucket_index);

hipError_t launch_moments(int storage, const void *I, const void *tab, const KParams &p,
                          void *E, void *F, hipStream_t s);
hipError_t launch_convert(const void *src, int src_storage, void *dst, int dst_storage,
                          const double *scales_dev, int ndir, int64_t ncell, hipStream_t s);
hipError_t launch_diag_reduce(const double *partials, int nblocks, double *diag,
                              int first_step, hipStream_t s);
hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t s);

}  // namespace lbrt
