// Internal types shared by the host dispatcher and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbrt.h"

namespace lbrt {

// 16-bit storage wrappers (bit patterns; conversions live in the kernels).
struct bf16_t { uint16_t u; };
struct f16_t { uint16_t u; };
// Equilibrium-shifted 16-bit storage: the deviation (I_i - w_i E) / s_i, with
// the cell's E in an FP32 array after the populations (KParams::e_off).
struct bf16s_t { uint16_t u; };
struct f16s_t { uint16_t u; };

// Per-direction constants, in processing order (antipodal pairs adjacent
// when the rule is centrally symmetric).  Axes where n^a == 0 get shift 0,
// so every tap of an in-box cell is an in-box address.
template <typename T>
struct DirTab {
  // The z-march reads two groups of fields per slot and plane, each laid out
  // contiguously so that it arrives in one or two wide scalar loads: the
  // interpolation and moment constants of the slot being streamed, and the
  // addresses of the slot whose loads are issued ahead.
  //
  // Weights per axis: wx = (1 - delta_x, delta_x), likewise wy; the z pair is
  // stored as (weight of the newly loaded plane, weight of the carried plane)
  // in the z-march order: (1 - delta_z, delta_z) when s_z >= 0,
  // (delta_z, 1 - delta_z) when s_z < 0.
  T wx[2], wy[2];
  T wz_new, wz_old;
  int32_t dzn;      // the new plane's z offset: 1 when s_z < 0, else 0
  int32_t active;   // 1 for a direction, 0 for a null (padding) slot
  T w;              // quadrature weight
  T n[3];           // unit direction
  T scale;          // storage scale s_i (1 for FP32/FP64)
  T inv_scale;      // 1 / s_i
  // Per-cell flux sums are formed against an isotropic reference (see the
  // step kernel): 1 / w (0 for a null slot), and the sum of n_i w_i over the
  // slots of the wave that owns this slot, in FP64 from the stored n and w.
  T invw;
  T dxs;            // delta_x * scale: x-face outflux per stored unit
  // Addresses: byte offsets of the direction's plane and of its y-halo row
  // (-sy * nx cells), the sx > 0 / sx < 0 all-ones/zero masks that pick the
  // lane's x-shifted offset, and dzn again (so that the group is one load).
  int64_t plane_off;// plane * ncell * size
  int64_t row_off;  // row_shift * size
  uint32_t mxp, mxm;
  int32_t dzn_a;
  int32_t row_shift;// -sy * nx
  // sx > 0 / sx < 0 as 0/1 factors (x-face tiles)
  T cxp, cxm;
  int64_t plane_el; // element offset of the direction's plane: plane * ncell
  double nwq[3];
  T tw[8];          // trilinear tap weights, tap b = bx | by << 1 | bz << 2 (eq. interp)
  T delta[3];       // dt |n^a| / dx, the fraction pulled from the upwind cell
  int32_t s[3];     // shift signs sgn(n^a), 0 where n^a == 0
  int32_t plane;    // storage plane (direction index in the caller's order)
  // Pair kernels, 16-bit storage: byte selector of v_perm_b32 that forms the
  // x-shifted pair of cells from the lane's own pair and its neighbouring
  // pair (sx > 0: (neighbour.hi, own.lo); otherwise (own.hi, neighbour.lo)).
  uint32_t psel;
  // Stochastic rounding of 16-bit storage: a random 32-bit constant of the
  // direction's storage plane (the element's random bits are this, the
  // cell's hash and the step's seed, combined by exclusive or).
  uint32_t rnd;
};

// Compact per-slot records of the pair kernel, read once per plane with one
// wide scalar load each (the full DirTab of 112 slots outgrows the scalar
// cache): the streaming phase's constants, and the collision's.
struct PairTab {                     // 64 bytes
  float wx0, wx1, wy0, wy1;          // per-axis interpolation weights (eq. interp)
  float wz_new, wz_old;              // z weights in march order (see DirTab)
  float w, invw;                     // quadrature weight and 1 / w (0 for a null slot)
  float n0, n1, n2;                  // unit direction
  float scale;                       // storage scale s_i (1 for FP32)
  int64_t plane_off;                 // byte offset of the direction's plane
  int32_t row_off;                   // byte offset of the y-halo row (-sy nx cells)
  uint32_t flags;                    // kPairSxPos | kPairDzn | kPairActive
};
struct PairColl {                    // 32 bytes
  float w, n0, n1, n2;
  float inv_scale;                   // 1 / s_i
  uint32_t rnd;                      // the plane's stochastic-rounding constant
  int64_t plane_off;
};
static_assert(sizeof(PairTab) == 64 && sizeof(PairColl) == 32,
              "one wide scalar load per record");
enum : uint32_t {
  kPairSxPos = 1u << 0,              // sx > 0: the x-shifted taps lie at x - 1
  kPairDzn = 1u << 1,                // sz < 0: the new plane is the one above
  kPairActive = 1u << 2,             // a direction (not a padding slot)
};

// A tile of the general (checked) path: 64 cells in a 2^txlog x 2^(6-txlog)
// xy block at (x0, y0), cells outside [x0, xe) x [y0, ye) inactive, marched
// over z planes [zb, ze).
struct GenTile {
  int32_t x0, y0, zb, ze;
  int32_t xe, ye, txlog, pad;
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

// The same table in compact form, passed by value as a kernel argument to
// the kernel that writes InflowArgs into device memory (a kernel node, so a
// step with inflow planes can be captured in a graph): the call's planes,
// and for each processing slot and axis the index of its plane or -1.
struct InflowCompact {
  int32_t n;
  int32_t face[LBRT_MAX_INFLOW];
  int32_t dir[LBRT_MAX_INFLOW];
  const float *ptr[LBRT_MAX_INFLOW];
  int8_t slot_plane[LBRT_MAX_DIRS][3];
};

// Waves per block of the step kernels (the wave q owns direction slots
// [q NB / waves, (q + 1) NB / waves)).
constexpr int waves_for(int nb) { return nb >= 112 ? 8 : 4; }

enum : uint32_t {
  KF_PAIRED = 1u << 0,   // directions come in antipodal pairs (2k, 2k+1)
  KF_MOVING = 1u << 1,   // mixed-frame collision (App. B)
  KF_DIAG = 1u << 2,     // per-block sums of E and E* into partials
  KF_WRITE_EF = 1u << 3, // write E, F of the new state
  KF_LAMZERO = 1u << 4,  // lambda == 0 (anisotropic term skipped)
  KF_XGHOSTS = 1u << 5,  // some inflow ghost plane sits on an x face
  KF_NWQZERO = 1u << 6,  // every wave's sum of n_i w_i is exactly 0
  KF_STOCH = 1u << 7,    // 16-bit storage rounds stochastically (seed below)
};

struct KParams {
  int32_t nx, ny, nz;
  int32_t ndir;
  int64_t ncell;
  int32_t tx, ty;              // xy tile in cells (tx * ty == 64, tx a power of two)
  int32_t txlog;               // log2(tx)
  int32_t ntx, nty;            // tiles per axis
  int32_t zlen;                // z-planes marched by one block of the main kernel
  // Main kernel tiles: x tiles [0, ntx), y tiles [main_ty0, main_ty0 + main_nty),
  // z ranges [main_zr0, main_zr0 + main_nzr); nblocks = ntx * main_nty * main_nzr.
  int32_t main_ty0, main_nty, main_zr0, main_nzr;
  int32_t nblocks;
  // General kernel: one block per GenTile entry.
  int32_t ngeneral;
  const GenTile *general_list;
  // Pair kernel (two x cells per lane) in place of the main kernel: tiles of
  // 128 cells at x0 = 128 k (k < ntx) computing the cells x in
  // [pair_x0, pair_xend) of rows [main_ty0, main_ty0 + main_nty), the same z
  // ranges.
  int32_t pair;
  int32_t pair_x0, pair_xend;
  // equilibrium-shifted storage: byte offset of a state's FP32 E array
  int64_t e_off;
  const PairTab *pair_tab;     // the pair kernel's slot records (nb of each)
  const PairColl *pair_coll;
  int32_t periodic[3];         // per axis x, y, z
  int32_t mode;                // lbrt_collision
  int32_t lambda_iters;
  uint32_t flags;
  uint32_t seed;               // this step's random seed (KF_STOCH)
  double dt;
  double lam;
};

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;   // waves per block = direction quarters
constexpr int kTileCells = 64;        // cells per xy tile (one per lane)
// E cells a block of equilibrium-shifted storage stages per plane: the
// tile and its one-cell halo, (64 / tx + 2)(tx + 2) <= 198, one per lane of
// four waves
constexpr int kStagePos = 256;
constexpr int kDiag = LBRT_DIAG_LEN;
// Per-block diagnostic partials of the step kernel: sum E, sum E*, outflux
// through the faces -x, +x, -y, +y, -z, +z, influx from inflow ghosts.
constexpr int kStepPartials = 9;
// Direction groups of the z-face flux kernel (its grid's second dimension).
constexpr int kZfaceGroups = 8;

// Direction-count buckets with a compiled kernel (multiples of 8: four waves
// times pairs).  Rules whose size is not a bucket run in the next larger
// bucket, padded with null directions.
constexpr int kBuckets[] = {16, 32, 56, 112, 152, 200};
constexpr int kNumBuckets = sizeof(kBuckets) / sizeof(kBuckets[0]);

// Launchers, one per (storage, bucket), defined in lbrt_step_*.hip.
using StepLauncher = hipError_t (*)(const void *Iin, void *Iout, const float *ka,
                                    const float *ks, const float *eta, const float *vel,
                                    const void *tab, const KParams &p,
                                    const InflowArgs *inflow, void *E, void *F,
                                    double *partials, hipStream_t s);

StepLauncher step_launcher(int storage, int bucket_index, bool moving);
// Whether the step launcher of (storage, bucket size, fluid) has the pair
// kernel (KParams::pair).
bool pair_available(int storage, int nb, bool moving);

// ---------------------------------------------------------------------------
// Batched form (one persistent launch over many domains)
// ---------------------------------------------------------------------------
// Buffers of a batch domain are byte offsets from the batch's global base
// pointer (a kernel argument), and its direction table an offset into the
// batch's table block (a read-only kernel argument): pointers read from
// device memory would make the compiler fall back to flat accesses and
// per-lane table loads.
constexpr int64_t kNoBuffer = INT64_MIN;
struct BatchDomain {
  KParams p;              // the domain's parameters (no diagnostics)
  int64_t tab;            // its direction table: byte offset into the table block
  int64_t I[2];           // ping-pong pair: step s reads I[s & 1]
  int64_t ka, ks, eta, vel;
  int64_t E, F;           // moments after the last step, or kNoBuffer
  const int4 *tiles;      // (x0, y0, zb, ze): the nmain main-path tiles
  const GenTile *gtiles;  // the general-path tiles
  int32_t ntiles, nmain;
  int32_t nsteps;
};

struct BatchPlan {
  const BatchDomain *dom;          // sorted by step count, longest first
  const long long *main_prefix;    // [ndom + 1]: main-path tiles of the first k domains
  const long long *gen_prefix;     // [ndom + 1]: general-path tiles of the first k domains
  const int32_t *step_active;      // [maxsteps]: domains active at step s (a prefix)
  int32_t maxsteps;
  const InflowArgs *noinflow;      // no ghost planes
  const char *tabs;                // the domains' direction tables
  char *gbase;                     // base of the domains' buffer offsets
};

// Launches steps [0, maxsteps) of a batch: per step, one launch of
// step_gen[s] general-path blocks and one of step_main[s] main-path blocks
// (host arrays).
using BatchLauncher = hipError_t (*)(const BatchPlan &bp, const long long *step_main,
                                     const long long *step_gen, hipStream_t s);
// The batched kernel for (storage, bucket, fluid), or nullptr.
BatchLauncher batch_launcher(int storage, int bucket_index, bool moving);


hipError_t launch_moments(int storage, const void *I, const void *tab, const KParams &p,
                          void *E, void *F, hipStream_t s);

// One direction of the coupling pass: n, the six products n_a n_b (xx, xy,
// xz, yy, yz, zz) and the storage scale, all FP64 (80 bytes).
struct CoupDir {
  double n[3];
  double nn[6];
  double s;
  double w;   // quadrature weight (equilibrium-shifted storage: I_i = w_i E + s_i d_i)
};
static_assert(sizeof(CoupDir) == 88, "CoupDir layout");

// Outputs (any may be null), the fluid inputs and the sizes of a coupling pass.
struct CoupArgs {
  void *E, *F, *P, *J, *H, *S;
  const float *vel, *kappa_a, *kappa_s, *eta;
  double ks_factor;   // 1 - lambda / 9: k_s = k_0 - k_1 / 3 with k_1 = lambda k_0 / 3
  int64_t ncell;
  int64_t e_off;      // equilibrium-shifted storage: byte offset of the state's E
  int ndir;
};
hipError_t launch_coupling(int storage, const void *I, const CoupDir *dir, const CoupArgs &a,
                           hipStream_t s);
hipError_t launch_convert(const void *src, int src_storage, void *dst, int dst_storage,
                          const double *scales_dev, const double *weights_dev, int ndir,
                          int64_t ncell, int64_t e_off, hipStream_t s);
// Reduces the step kernel's per-block partials (nblocks rows of
// kStepPartials) into diag in a fixed order: sums of E and E* replace diag[0]
// and diag[8]; fluxes are added to diag[1..7] (replaced when first_step).
hipError_t launch_diag_reduce(const double *partials, int nblocks, double *diag, int first_step,
                              hipStream_t s);
hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t s);
// Streaming copy of n16 16-byte elements (the measured bandwidth ceiling).
hipError_t launch_stream_copy(const void *src, void *dst, int64_t n16, hipStream_t s);
// Writes the ghost-plane table described by c into *out (one small block).
hipError_t launch_inflow_table(const InflowCompact &c, InflowArgs *out, hipStream_t s);
// Adjoint of one step (FP32 or FP64 storage): nu is a work buffer of one
// state; gradients are added into g_ka, g_ks, g_eta.
hipError_t launch_adjoint(int storage, const void *I, const void *lam_next, void *lam_out,
                          void *nu, int face, void *g_ka, void *g_ks, void *g_eta,
                          const float *ka, const float *ks, const float *eta, const float *vel,
                          const void *tab, const KParams &p, const InflowArgs *inflow,
                          hipStream_t s);
// Blocks of the z-face flux kernel (0 on a periodic z axis), and its launch:
// per-block partials in the step kernel's format.
int zface_blocks(const KParams &p);
hipError_t launch_zface(int storage, const void *I, const void *tab, const KParams &p,
                        const InflowArgs *inflow, double *partials, hipStream_t s);

}  // namespace lbrt
