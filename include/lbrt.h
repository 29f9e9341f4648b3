/*
 * lbrt — fused stream-and-collide step of the grey radiative-transfer
 * lattice-Boltzmann scheme of Weih, Gabbana, Simeoni, Rezzolla, Succi and
 * Tripiccione (2020), for AMD MI355X (gfx950).
 *
 * One step (Sec. 3.3 "Numerical procedure") does, for every cell r and
 * discrete direction n_i:
 *   stream   I*_i(r) = I_i(r - n_i dt), by the trilinear interpolation of
 *            eq. (interp) from the 2x2x2 upwind cells;
 *   moments  E* = sum_i I*_i, F* = sum_i n_i I*_i (eq. moments_discrete);
 *   collide  relax toward the isotropic equilibrium w_i (E + lambda n_i.F)
 *            with absorption kappa_a, emission eta and scattering kappa_s
 *            (eqs. rte_gray_bgkform, source-and-equil), implicitly
 *            (eq. rte_implicit), explicitly (eq. collision-step) or by a
 *            fixed number of Lambda-iteration cycles; or, for a moving
 *            fluid, the implicit mixed-frame equation of App. B.
 *
 * Conventions shared by every entry point
 *   - Uniform Cartesian grid nx * ny * nz, spacing dx; cell (x, y, z) has
 *     linear index x + nx * (y + ny * z).
 *   - Populations are weight-absorbed, I_i = w_i I(n_i) (Sec. 3.2), stored
 *     structure-of-arrays, direction-major: element (i, cell) at
 *     i * ncell + cell, in the context's storage type.  BF16 and FP16
 *     storage hold I_i / s_i with a per-direction scale s_i (default |w_i|).
 *   - Per-cell coefficient fields are float32 arrays of ncell values.
 *     kappa_s is the isotropic scattering coefficient kappa_0 of
 *     eq. (rte_gray); lambda = 3 kappa_1 / kappa_0 is a scalar of the context.
 *     With a moving fluid, kappa_a, kappa_s and eta are fluid-frame values and
 *     vel holds (vx[ncell], vy[ncell], vz[ncell]) in units of c.
 *   - Device pointers are plain HIP device addresses owned by the caller;
 *     the library never frees them.  Work is enqueued on the caller's HIP
 *     stream (a hipStream_t passed as void*, NULL = default stream) and is
 *     asynchronous; errors detected on the host are returned before any
 *     launch.  Every call returns an lbrt_status code and never aborts;
 *     lbrt_last_error() gives a message for the calling thread.
 *   - A context owns work memory that its calls reuse (diagnostic partials,
 *     the inflow ghost table, the adjoint's work state).  Calls on one
 *     context must therefore be ordered: issue them on one stream, or
 *     synchronise between streams.  Calls on different contexts are
 *     independent.
 */
#ifndef LBRT_H
#define LBRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbrt_ctx lbrt_ctx;

typedef enum {
  LBRT_OK = 0,
  LBRT_E_INVAL = -1,        /* bad argument: null pointer, bad size or enum     */
  LBRT_E_CFL = -2,          /* dt > dx: the 2x2x2 stencil spans one cell only   */
  LBRT_E_QUAD = -3,         /* directions/weights violate the rule identities   */
  LBRT_E_NOMEM = -4,        /* device allocation for the context tables failed  */
  LBRT_E_HIP = -5,          /* a HIP runtime call failed                        */
  LBRT_E_UNSUPPORTED = -6   /* valid but not supported combination              */
} lbrt_status;

typedef enum { LBRT_BC_OUTFLOW = 0, LBRT_BC_PERIODIC = 1, LBRT_BC_INFLOW = 2 } lbrt_bc;
/* Population storage.  The equilibrium-shifted forms store the deviation
 * d_i = (I_i - w_i E) / s_i of each population from the cell's isotropic
 * equilibrium in BF16 or FP16, and the cell's E in FP32 after them: a state
 * is ndir * ncell 16-bit values, then (at byte lbrt_state_e_offset, the
 * first multiple of 256 at or after 2 ndir ncell) ncell float32 values; its
 * size is lbrt_state_bytes.  In optically thick cells I_i is close to
 * w_i E, and the deviation keeps F (a small difference of populations of
 * size w_i E) to the 16-bit format's relative precision.  Static fluid only;
 * the interior runs on the one-cell-per-lane kernel. */
typedef enum {
  LBRT_FP32 = 0,
  LBRT_FP64 = 1,
  LBRT_BF16 = 2,
  LBRT_FP16 = 3,
  LBRT_BF16_SHIFTED = 4,
  LBRT_FP16_SHIFTED = 5
} lbrt_storage;
/* Rounding of populations stored as BF16/FP16 (ignored for FP32/FP64). */
typedef enum {
  LBRT_ROUND_STOCHASTIC = 0, /* round up with the probability of the dropped
                                fraction: exact in expectation              */
  LBRT_ROUND_NEAREST = 1     /* round to nearest even                         */
} lbrt_rounding;
typedef enum {
  LBRT_COLL_IMPLICIT = 0,   /* eq. (rte_implicit), solved exactly                */
  LBRT_COLL_EXPLICIT = 1,   /* eq. (collision-step)                              */
  LBRT_COLL_LAMBDA = 2      /* Lambda iteration, lambda_iters cycles (Sec. 3.3)  */
} lbrt_collision;

enum { LBRT_MAX_DIRS = 200, LBRT_MAX_INFLOW = 32, LBRT_DIAG_LEN = 9 };

/* Face order used by bc[], inflow planes and diagnostics. */
enum { LBRT_FACE_MX = 0, LBRT_FACE_PX = 1, LBRT_FACE_MY = 2, LBRT_FACE_PY = 3,
       LBRT_FACE_MZ = 4, LBRT_FACE_PZ = 5 };

/*
 * Problem statement (Sec. 3.2-3.3; boundaries Sec. 4.1.1 and 4.2.1).
 *   dirs     host, ndir x 3 unit vectors n_i (row i = (nx, ny, nz));
 *   weights  host, ndir nonzero quadrature weights, sum 1 (Sec. 3.2.1; some
 *            Lebedev rules carry negative weights);
 *   scale    host, ndir per-direction storage scales s_i > 0 for BF16/FP16,
 *            or NULL for s_i = |w_i|; ignored for FP32/FP64;
 *   bc       per face: outflow (vacuum ghosts, nothing enters), periodic
 *            (both faces of an axis), or inflow (ghost values given per step
 *            as lbrt_inflow planes; ghosts not given are vacuum);
 *   lambda_iters  cycles for LBRT_COLL_LAMBDA (>= 1);
 *   lambda_aniso  lambda = 3 kappa_1 / kappa_0 (0 for isotropic scattering);
 *   moving_fluid  nonzero: lbrt_step takes a velocity field and uses the
 *            mixed-frame collision of App. B (implicit, lambda must be 0);
 *   rounding BF16/FP16 storage: LBRT_ROUND_STOCHASTIC (0, the default) or
 *            LBRT_ROUND_NEAREST.  Round-to-nearest loses every per-step
 *            change below half a unit in the last place (2^-9 relative for
 *            BF16, 2^-12 for FP16), so a weakly absorbing cell never dims a
 *            beam; stochastic rounding is unbiased.  Its random bits per
 *            element are a hash of the cell index and a per-step seed (drawn
 *            from the context's count of steps taken), combined with a
 *            constant of the direction, so a run on a fresh context is
 *            reproducible (a captured graph replays the seeds it captured).
 * The context copies everything it needs; the caller's arrays may be freed
 * after lbrt_init returns.
 */
typedef struct {
  int32_t nx, ny, nz;
  double dx, dt;
  int32_t ndir;
  const double *dirs;
  const double *weights;
  const double *scale;
  int32_t bc[6];
  int32_t storage;
  int32_t collision;
  int32_t lambda_iters;
  double lambda_aniso;
  int32_t moving_fluid;
  int32_t rounding;
} lbrt_desc;

/*
 * Prescribed ghost values for direction `dir` on inflow face `face`
 * (the beam injection of Sec. 4.1.1).  `values` is a device float32 array
 * in the face's own layout: x faces [z][y], y faces [z][x], z faces [y][x].
 * It is read when a population streams in through that face: only
 * directions that enter through the face may be listed.
 */
typedef struct {
  int32_t face;
  int32_t dir;
  const float *values;
} lbrt_inflow;

/* Bytes of one state buffer of a problem: ndir * ncell elements of the
 * storage type, plus the E array for the equilibrium-shifted forms; and the
 * byte offset of that E array (0 for the other forms).  Host only; -1 for a
 * storage value that is not a storage type. */
int64_t lbrt_state_bytes(int32_t storage, int32_t ndir, int64_t ncell);
int64_t lbrt_state_e_offset(int32_t storage, int32_t ndir, int64_t ncell);

/* Host-only check of a problem statement; needs no GPU.  Rejects
 * dt <= 0 or dt > dx (LBRT_E_CFL), dims < 2, ndir outside [2, LBRT_MAX_DIRS],
 * non-unit directions, |sum w - 1|, |sum w n|, |sum w n n - I/3| > 1e-12
 * (LBRT_E_QUAD: the collision relies on these identities, App. A.1
 * eq. stencil-symmetry), a periodic flag on one face of an axis only,
 * bad enums, negative scales, lambda_iters < 1 in Lambda mode, and
 * moving_fluid with lambda != 0 or a non-implicit collision. */
int lbrt_validate(const lbrt_desc *desc);

/* Validate, then build a context on the current HIP device: direction and
 * stencil tables in device memory, a small reduction buffer for the
 * diagnostics, kernel selection.  *out is set only on success.
 * Environment variables read here change speed only, never results:
 * LBRT_TILE ("TXxTY", tx * ty = 64) and LBRT_ZLEN, LBRT_ZLEN_GENERAL (z-range
 * lengths) set the initial tiling (see lbrt_set_tiling); LBRT_FP64_FLUX_TERM
 * (any value) keeps the FP64 reference term of the per-cell flux sums where
 * it is exactly zero (rules whose antipodal pairs share a wave); LBRT_PAIR=0
 * runs the interior on the one-cell-per-lane kernel instead of the
 * two-cells-per-lane one. */
int lbrt_init(const lbrt_desc *desc, lbrt_ctx **out);

/* Free the context's device tables.  NULL is accepted. */
void lbrt_destroy(lbrt_ctx *ctx);

/*
 * nsteps >= 0 stream-collide steps.  Step k reads I_a (k even) or I_b
 * (k odd) and writes the other buffer (ping-pong; in-place is rejected):
 * the result is in I_b when nsteps is odd, in I_a otherwise.  With
 * nsteps = 0 the state is left as it is, E and F (if given) get the
 * moments of I_a and diag (if given) is zeroed.
 *   kappa_a, kappa_s, eta  required (device float32, ncell each);
 *   vel      device float32 3 x ncell, required iff moving_fluid;
 *   inflow   host array of ninflow planes (ninflow <= LBRT_MAX_INFLOW), or
 *            NULL/0; each plane must name an inflow face and a direction
 *            entering through it;
 *   E, F     device, or NULL: moments of the final state, E[ncell] and
 *            F[3][ncell] (x, y, z components), float64 for FP64 storage and
 *            float32 otherwise;
 *   diag     device float64[LBRT_DIAG_LEN], or NULL:
 *            [0] sum over cells of E after the last step,
 *            [1..6] energy streamed out through faces -x,+x,-y,+y,-z,+z,
 *                   summed over the call's steps (a point outside along
 *                   several axes is booked on the first of x, y, z),
 *            [7] energy streamed in from inflow ghosts, summed over steps,
 *            [8] sum over cells of the streamed E* of the last step.
 *            diag is overwritten by the call.
 * The call enqueues kernels only (the ghost-plane table is written by a
 * kernel from the call's arguments), so it can be captured in a HIP graph,
 * except for a call with diag that first grows the context's partials
 * buffer (one hipMalloc when the tiling needs more rows than lbrt_init
 * sized; lbrt_step_noalloc never allocates).
 */
int lbrt_step(lbrt_ctx *ctx, void *I_a, void *I_b,
              const float *kappa_a, const float *kappa_s, const float *eta,
              const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
              int32_t nsteps, void *E, void *F, double *diag, void *stream);

/*
 * lbrt_step without allocation, for callers that cannot call hipMalloc:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Arguments, results and errors are those of lbrt_step (the
 * same kernels, bit-identical results).  The work memory (the ghost-plane
 * table and the per-block diagnostic partials) is a fixed 4 MiB array in
 * device memory, one per GPU, held until the process ends; the call
 * allocates nothing and copies nothing from the host (the ghost table is
 * written by a kernel from its arguments).  With diag != NULL the call
 * needs one 72-byte partial row per step-kernel block plus the z-face
 * blocks; more than the array holds (about 58,000 rows: 256^3 with the
 * default tiling needs about 13,000) is rejected with LBRT_E_INVAL before
 * any launch.  The context's device must be the current device.
 * Every call on one GPU uses that GPU's array: calls that can overlap on
 * one GPU (different streams, or host threads, without ordering) race.
 */
int lbrt_step_noalloc(lbrt_ctx *ctx, void *I_a, void *I_b,
                      const float *kappa_a, const float *kappa_s, const float *eta,
                      const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
                      int32_t nsteps, void *E, void *F, double *diag, void *stream);

/*
 * Adjoint of one step, for the reverse sweep of a run whose objective is
 *   L = sum over the states I^n entering the run's steps of the energy that
 *       streams out through face detector_face (diag[1 + face] of lbrt_step).
 * Not in the paper: the exact transpose of its implicit step (Sec. 3.3, and
 * App. B for a moving fluid), which is linear in the populations.  For step
 * n (I^(n+1) = C(S I^n), S the pull of eq. (interp), C the collision):
 *   lam_out   = d + S^T (dC/dI*)^T lam_next   (d: detector weights on the face),
 *   g_*      += (dC/d field)^T lam_next       per cell.
 *   I_n       device, the state entering the forward step (storage type);
 *   lam_next  device, adjoint of the state after the step (same type; zero
 *             for the last step); lam_out receives the adjoint of I_n and
 *             must not overlap lam_next;
 *   detector_face  0..5 (-x,+x,-y,+y,-z,+z), or -1 for no detector term;
 *   g_kappa_a, g_kappa_s, g_eta  device, ncell each, float64 for FP64
 *             storage and float32 otherwise; the step's gradients are ADDED;
 *   kappa_a, kappa_s, eta, vel, inflow  the forward step's inputs (the inflow
 *             ghosts fix the point of linearisation only).
 * Supported: FP32 and FP64 storage, the implicit collision with lambda = 0,
 * static or moving fluid (else LBRT_E_UNSUPPORTED).  The first call
 * allocates a context-owned work buffer of one state.
 */
int lbrt_adjoint_step(lbrt_ctx *ctx, const void *I_n, const void *lam_next, void *lam_out,
                      int32_t detector_face, void *g_kappa_a, void *g_kappa_s, void *g_eta,
                      const float *kappa_a, const float *kappa_s, const float *eta,
                      const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
                      void *stream);

/* Moments E = sum_i I_i and F = sum_i n_i I_i (eq. moments_discrete) of a
 * stored state I; E, F as in lbrt_step (either may be NULL). */
int lbrt_moments(lbrt_ctx *ctx, const void *I, void *E, void *F, void *stream);

/*
 * Outputs of lbrt_coupling, each a device array (NULL: not computed), in
 * float64 for FP64 storage and float32 otherwise, component-major like F:
 *   E  ncell      E = sum_i I_i                           (eq. moments_discrete)
 *   F  3 x ncell  F^j = sum_i n_ij I_i
 *   P  6 x ncell  P^xx, P^xy, P^xz, P^yy, P^yz, P^zz,
 *                 P^jk = sum_i n_ij n_ik I_i              (eq. higher_moments)
 *   J  ncell      fluid-frame energy density
 *                 W^2 (E - 2 F.v + v.P.v)                 (eq. J)
 *   H  4 x ncell  H_0, H_x, H_y, H_z: fluid-frame flux,
 *                 H_j = W^3 (F.v - E) v_j + W h_ji (F^i - P^ik v_k),
 *                 h_ij = W^2 v_i v_j + delta_ij            (eq. J);
 *                 H_0 = v.H, the time component orthogonal to the fluid
 *                 four-velocity (taken so that S_0 is the energy the
 *                 collision takes from the radiation)
 *   S  4 x ncell  S_0 = W (kappa_a J - eta) + k H_0,
 *                 S_j = W (kappa_a J - eta) v_j + k H_j,
 *                 k = kappa_a + kappa_s - kappa_1 / 3 with
 *                 kappa_1 = lambda kappa_s / 3       (Sec. 5, coupling item 4)
 */
typedef struct {
  void *E, *F, *P, *J, *H, *S;
} lbrt_coupling_out;

/* What the coupling loop of Sec. 5 (items 3 and 4) takes from a state I
 * (storage type of the context) after a step: the lab-frame moments, the
 * fluid-frame J and H, and the radiative sources, per cell, with every sum
 * over directions in FP64.
 *   vel      device, 3 x ncell float32 fluid velocity in units of c,
 *            |v| < 1 (else the results are not finite); NULL: at rest;
 *   kappa_a, kappa_s, eta  device, ncell float32 fluid-frame fields; needed
 *            only for S (else LBRT_E_INVAL), may be NULL otherwise;
 *   out      host struct of output pointers; outputs must not overlap I or
 *            each other.
 * The sources use lambda from the context.  One launch on `stream`; no
 * allocation, so it may be captured in a graph. */
int lbrt_coupling(lbrt_ctx *ctx, const void *I, const float *vel, const float *kappa_a,
                  const float *kappa_s, const float *eta, const lbrt_coupling_out *out,
                  void *stream);

/* Convert a population array between storage types with the context's
 * per-direction scales (e.g. to encode an initial state for BF16/FP16
 * storage, or decode one for inspection).  src and dst must not overlap. */
int lbrt_convert(lbrt_ctx *ctx, const void *src, int32_t src_storage,
                 void *dst, int32_t dst_storage, void *stream);

/*
 * Tiling of a context's step kernels: xy tiles of tx x ty cells (tx * ty = 64,
 * tx a power of two) and z ranges of zlen planes (main kernel) and
 * zlen_general planes (boundary tiles).  Tiling changes speed only: results
 * are bit-identical for every choice.  The autotuner calls this.
 */
int lbrt_set_tiling(lbrt_ctx *ctx, int32_t tx, int32_t ty, int32_t zlen, int32_t zlen_general);

/* The context's current tiling (the defaults chosen by lbrt_init from the grid
 * shape, or the last lbrt_set_tiling).  Any output pointer may be NULL.
 * Errors: LBRT_E_INVAL when ctx is NULL. */
int lbrt_get_tiling(const lbrt_ctx *ctx, int32_t *tx, int32_t *ty, int32_t *zlen,
                    int32_t *zlen_general);

/*
 * Batched form: many independent domains (each its own context, buffers,
 * fields and step count) advanced together.  Not in the paper.  A domain runs
 * nsteps steps as lbrt_step would (result in I_b when nsteps is odd), without
 * diagnostics or inflow ghosts; E, F (or NULL) receive its moments after the
 * last step.  Every domain must share the storage type, the direction bucket
 * and the fluid kind of the first; supported: FP32 storage, static fluid.
 * Step s of the batch is two kernel launches (boundary tiles, then interior
 * tiles) over every tile of every domain still running at step s, so small
 * domains fill the GPU together.
 *
 * lbrt_batch_create builds the tile lists on the host and uploads them (call
 * it outside graph capture); the domains' contexts and buffers must outlive
 * the batch.  lbrt_step_batched only enqueues kernels (two per step of the
 * longest domain) and may be captured in a hipGraph and replayed as one.
 */
typedef struct {
  lbrt_ctx *ctx;
  void *I_a, *I_b;
  const float *kappa_a, *kappa_s, *eta, *vel;
  int32_t nsteps;
  void *E, *F;
} lbrt_domain;

typedef struct lbrt_batch lbrt_batch;

int lbrt_batch_create(const lbrt_domain *domains, int32_t ndomains, lbrt_batch **out);
int lbrt_step_batched(lbrt_batch *batch, void *stream);
void lbrt_batch_destroy(lbrt_batch *batch);

/* A plain streaming copy of `bytes` (a multiple of 16; 16-byte aligned,
 * non-overlapping device buffers): 16-byte loads and non-temporal stores.
 * Not part of the method: the measured read-plus-write bandwidth ceiling
 * that the step kernels are compared with. */
int lbrt_stream_copy(const void *src, void *dst, int64_t bytes, void *stream);

/* Message describing the last error returned on the calling thread
 * (empty string if none).  The pointer stays valid until the thread's next
 * lbrt call. */
const char *lbrt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBRT_H */
