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
// when the rule is centrally symmetric).  Axes where n^a == 0 get shift 0,
// so every tap of an in-box cell is an in-box address.
template <typename T>
struct DirTab {
  T tw[8];          // trilinear tap weights, tap b = bx | by << 1 | bz << 2 (eq. interp)
  int32_t off[8];   // byte offset of tap b from its cell: -(bx sx + by sy nx + bz sz nx ny) * size
  int64_t plane_off;// byte offset of the direction's plane: plane * ncell * size
  T w;              // quadrature weight
  T n[3];           // unit direction
  T delta[3];       // dt |n^a| / dx, the fraction pulled from the upwind cell
  T scale;          // storage scale s_i (1 for FP32/FP64)
  T inv_scale;      // 1 / s_i
  int32_t s[3];     // shift signs sgn(n^a), 0 where n^a == 0
  int32_t plane;    // storage plane (direction index in the caller's order)
};

// Inflow ghost planes of one call, kept in device memory (context-owned) so
// that kernels index it with scalar loads.
struct InflowArgs {
  int32_t n;
  int32_t face[LBRT_MAX_INFLOW];
  int32_t dir[LBRT_MAX_INFLOW];      // storage plane index
  const float *ptr[LBRT_MAX_INFLOW];
  // For processing slot k and axis a: the ghost plane that slot pulls from
  // along a (the low face when s_a > 0, the high face when s_a < 0), or null.
  const float *ghost[LBRT_MAX_DIRS][3];
};

enum : uint32_t {
  KF_PAIRED = 1u << 0,   // directions come in antipodal pairs (2k, 2k+1)
  KF_MOVING = 1u << 1,   // mixed-frame collision (App. B)
  KF_DIAG = 1u << 2,     // per-block sums of E and E* into partials
  KF_WRITE_EF = 1u << 3, // write E, F of the new state
  KF_LAMZERO = 1u << 4,  // lambda == 0 (anisotropic term skipped)
  KF_XGHOSTS = 1u << 5,  // some inflow ghost plane sits on an x face
};

struct KParams {
  int32_t nx, ny, nz;
  int32_t ndir;
  int64_t ncell;
  int32_t tx, ty, tz;          // tile shape in cells (tx * ty * tz == 64)
  int32_t ntx, nty, ntz;       // tiles per axis
  int32_t ntiles;
  int32_t slab;                // y-blocks per slab of the tile sweep
  int32_t periodic[3];         // per axis x, y, z
  int32_t mode;                // lbrt_collision
  int32_t lambda_iters;
  uint32_t flags;
  double dt;
  double lam;
};

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;   // waves per block = direction quarters
constexpr int kTileCells = 64;        // cells per block tile (one per lane)
constexpr int kDiag = LBRT_DIAG_LEN;
constexpr int kStepPartials = 2;   // per block: sum E, sum E*
constexpr int kFacePartials = 7;   // per block: outflux on 6 faces, influx

// Direction-count buckets with a compiled kernel (multiples of 8: four waves
// times pairs).  Rules whose size is not a bucket run in the next larger
// bucket, padded with null directions.
constexpr int kBuckets[] = {16, 32, 56, 64, 112, 128, 152, 160};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);

// Launchers, one per (storage, bucket), defined in lbrt_step_*.hip.
using StepLauncher = hipError_t (*)(const void *Iin, void *Iout, const float *ka,
                                    const float *ks, const float *eta, const float *vel,
                                    const void *tab, const KParams &p,
                                    const InflowArgs *inflow, void *E, void *F,
                                    double *partials, hipStream_t s);

StepLauncher step_launcher(int storage, int bucket_index, bool moving);

hipError_t launch_moments(int storage, const void *I, const void *tab, const KParams &p,
                          void *E, void *F, hipStream_t s);
hipError_t launch_convert(const void *src, int src_storage, void *dst, int dst_storage,
                          const double *scales_dev, int ndir, int64_t ncell, hipStream_t s);
// Boundary fluxes of a state (outflux per face, inflow influx) into
// per-block partials; returns the number of blocks used in *nblocks.
hipError_t launch_face_flux(int storage, const void *I, const void *tab, const KParams &p,
                            const InflowArgs *inflow, double *partials, int *nblocks,
                            hipStream_t s);
int face_flux_blocks(const KParams &p);
hipError_t launch_diag_reduce(const double *step_partials, int step_blocks,
                              const double *face_partials, int face_blocks, double *diag,
                              int first_step, hipStream_t s);
hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t s);

}  // namespace lbrt
