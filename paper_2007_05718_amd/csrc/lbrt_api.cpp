// Host side of the C ABI: validation, context tables, kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbrt_internal.h"

using namespace lbrt;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(LBRT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t storage_bytes(int s) {
  switch (s) {
    case LBRT_FP32: return 4;
    case LBRT_FP64: return 8;
    default: return 2;
  }
}

bool is_shifted(int s) { return s == LBRT_BF16_SHIFTED || s == LBRT_FP16_SHIFTED; }
bool is_reduced(int s) {
  return s == LBRT_BF16 || s == LBRT_FP16 || is_shifted(s);
}

// Byte offset of the E array in an equilibrium-shifted state (0 otherwise)
// and the bytes of one state buffer.
int64_t e_offset(int s, int ndir, int64_t ncell) {
  if (!is_shifted(s)) return 0;
  return (2 * (int64_t)ndir * ncell + 255) / 256 * 256;
}
int64_t state_bytes(int s, int ndir, int64_t ncell) {
  if (is_shifted(s)) return e_offset(s, ndir, ncell) + 4 * ncell;
  return (int64_t)storage_bytes(s) * ndir * ncell;
}

struct TileShape { int tx, ty; };

// Device memory of lbrt_step_noalloc, for callers that cannot allocate: the
// ghost-plane table, then the per-block diagnostic partials.  One copy per
// GPU for the life of the process; every call on that GPU reuses it.
constexpr size_t kScratchBytes = (size_t)4 << 20;
constexpr size_t kScratchTableBytes = (sizeof(InflowArgs) + 255) / 256 * 256;
constexpr int kScratchMaxPartials =
    (int)((kScratchBytes - kScratchTableBytes) / (sizeof(double) * kStepPartials));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// scratch's device address on each GPU (hipGetSymbolAddress with that GPU
// current); host code passes these, never the array's name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

struct lbrt_ctx {
  lbrt_desc desc;                 // pointers in desc are not kept
  std::vector<double> dirs, weights, scales;
  int bucket = 0;                 // index into kBuckets
  int nb = 0;                     // bucket size
  bool paired = false;
  bool nwq_zero = false;          // every wave's sum of n_i w_i is exactly 0
  std::vector<int> order;         // processing index -> storage plane
  void *tab_dev = nullptr;        // DirTab<float> or DirTab<double>, nb entries
  size_t tab_bytes = 0;
  CoupDir *coup_dev = nullptr;    // the coupling pass's direction table
  double *scales_dev = nullptr;   // per storage plane
  double *weights_dev = nullptr;  // per storage plane (shifted storage conversions)
  double *partials = nullptr;     // per-block sums of the step kernel
  int partials_cap = 0;
  InflowArgs *inflow_dev = nullptr; // ghost-plane table of the current call
  bool any_inflow_face = false;     // some face is LBRT_BC_INFLOW
  void *adj_work = nullptr;         // one state: the adjoint's nu buffer
  TileShape tile{64, 1};
  int zlen = 64;                  // z-planes per block of the main kernel
  int zlen_general = 4;           // z-planes per block of the general kernel
  // Tile plans [mode][variant]: mode 0 runs the interior on the main kernel
  // (one cell per lane), mode 1 on the pair kernel (two x cells per lane);
  // variant 1 is for calls with inflow ghost planes on a z face.
  struct Plan {
    std::vector<GenTile> general;   // the general-path tiles
    GenTile *dev = nullptr;         // the same, on the device
    int zr0 = 0, nzr = 0;           // the main (or pair) kernel's z ranges
  } plan[2][2];
  bool pair = false;              // lbrt_step runs mode 1
  PairTab *pair_tab_dev = nullptr;   // the pair kernel's slot records (nb each)
  PairColl *pair_coll_dev = nullptr;
  uint64_t round_seq = 0;         // steps taken: the stochastic rounding seeds
  int device = 0;
  unsigned char *scratch = nullptr;  // this device's scratch (lbrt_step_noalloc)
};

namespace {

bool is_periodic_pair_ok(const int32_t *bc) {
  for (int a = 0; a < 3; ++a) {
    const bool lo = bc[2 * a] == LBRT_BC_PERIODIC, hi = bc[2 * a + 1] == LBRT_BC_PERIODIC;
    if (lo != hi) return false;
  }
  return true;
}

int bucket_for(int ndir) {
  for (int b = 0; b < kNumBuckets; ++b)
    if (kBuckets[b] >= ndir) return b;
  return -1;
}

TileShape default_tile(int nx, int ny, int nz) {
  if (const char *env = std::getenv("LBRT_TILE")) {
    TileShape t{};
    if (std::sscanf(env, "%dx%d", &t.tx, &t.ty) == 2 && t.tx > 0 && t.ty > 0 &&
        t.tx * t.ty == kTileCells && (t.tx & (t.tx - 1)) == 0)
      return t;
  }
  (void)ny;
  (void)nz;
  if (nx >= 64) return {64, 1};
  if (nx >= 32) return {32, 2};
  if (nx >= 16) return {16, 4};
  return {8, 8};
}

// z-planes marched by one block: long enough that the prologue plane (one
// extra plane per range) is cheap, short enough that the grid has several
// blocks per CU: about `target` blocks (main kernel: 8192, 32 per CU, measured
// fastest at 256^3; the pair kernel's blocks do twice the work: 4096), never
// fewer than 16 planes.
int default_zlen(int nz, int64_t xy_tiles, int64_t target) {
  if (const char *env = std::getenv("LBRT_ZLEN")) {
    const int v = std::atoi(env);
    if (v > 0) return v;
  }
  xy_tiles = std::max<int64_t>(xy_tiles, 1);
  int64_t ranges = (target + xy_tiles - 1) / xy_tiles;
  int zlen = (int)std::max<int64_t>(16, (nz + ranges - 1) / ranges);
  return std::min(zlen, nz);
}

// The pair kernel computes x in [2, nx - 2) of rows [1, ny - 1), in tiles of
// 128 cells at x = 128 k (whole cache lines).
constexpr int kPairX0 = 2;
constexpr int kPairTile = 128;
int pair_ntx(int nx) { return (nx + kPairTile - 1) / kPairTile; }
// With periodic x the two face columns at each end of a row are general
// (checked) tiles; otherwise the pair kernel computes the whole row.
bool pair_face_columns(const lbrt_desc &d) {
  return d.bc[LBRT_FACE_MX] == LBRT_BC_PERIODIC;
}

// A fixed random 32-bit constant per storage plane (splitmix64 of its index):
// one of the three parts of an element's stochastic rounding bits.
uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
uint32_t plane_random(int plane) { return (uint32_t)(splitmix64(0x6c627274u + plane) >> 32); }

// Direction table in processing order: nb slots (directions, then null
// slots), stored twice (the step kernel reads copy z & 1 on plane z).
template <typename T>
void build_table(const lbrt_ctx &c, std::vector<DirTab<T>> &tab) {
  const lbrt_desc &d = c.desc;
  tab.assign((size_t)c.nb, DirTab<T>{});
  const double dx = d.dx, dt = d.dt;
  const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
  const int64_t esize = (int64_t)storage_bytes(d.storage);
  for (int k = 0; k < c.nb; ++k) {
    DirTab<T> &e = tab[k];
    std::memset(&e, 0, sizeof(e));
    if (k >= d.ndir) {
      // null slot: reads in-box cells of plane order[0] with every weight 0,
      // so its streamed value is 0 and it adds nothing to the moments; it is
      // never stored (active = 0)
      e.plane = c.order[0];
      e.plane_el = (int64_t)e.plane * ncell;
      e.plane_off = (int64_t)e.plane * ncell * esize;
      e.scale = T(1);
      e.inv_scale = T(1);
      // a selector that merges two stored values (any other could assemble
      // a NaN bit pattern, and 0 * NaN is not 0)
      e.psel = 0x01000706u;
      continue;
    }
    const int i = c.order[k];
    const double *n = &c.dirs[3 * i];
    double delta[3];
    int s[3];
    for (int a = 0; a < 3; ++a) {
      // The pulled fraction on the working precision's grid (2^-24 for FP32,
      // 2^-53 for FP64): then 1 - delta is exact too, the two weights of an
      // axis sum to exactly 1 and the pull conserves energy up to unbiased
      // rounding (with 1 - delta rounded on its own, a drift of ~1e-8 per
      // step).
      const int bits = std::numeric_limits<T>::digits;
      delta[a] = std::ldexp(std::nearbyint(std::ldexp(dt * std::fabs(n[a]) / dx, bits)), -bits);
      s[a] = n[a] > 0.0 ? 1 : (n[a] < 0.0 ? -1 : 0);
      if (delta[a] == 0.0) s[a] = 0;
    }
    for (int b = 0; b < 8; ++b) {
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      const double wx = bx ? delta[0] : 1.0 - delta[0];
      const double wy = by ? delta[1] : 1.0 - delta[1];
      const double wz = bz ? delta[2] : 1.0 - delta[2];
      e.tw[b] = (T)(wx * wy * wz);
    }
    e.wx[0] = (T)(1.0 - delta[0]);
    e.wx[1] = (T)delta[0];
    e.wy[0] = (T)(1.0 - delta[1]);
    e.wy[1] = (T)delta[1];
    // z weights in march order: (new plane, carried plane)
    e.wz_new = (T)(s[2] < 0 ? delta[2] : 1.0 - delta[2]);
    e.wz_old = (T)(s[2] < 0 ? 1.0 - delta[2] : delta[2]);
    e.dxs = (T)(delta[0] * c.scales[i]);
    e.cxp = (T)(s[0] > 0 ? 1.0 : 0.0);
    e.cxm = (T)(s[0] < 0 ? 1.0 : 0.0);
    e.mxp = s[0] > 0 ? 0xffffffffu : 0u;
    e.mxm = s[0] < 0 ? 0xffffffffu : 0u;
    e.dzn = s[2] < 0 ? 1 : 0;
    e.dzn_a = e.dzn;
    e.active = 1;
    e.row_shift = -s[1] * d.nx;
    e.row_off = (int64_t)e.row_shift * esize;
    e.w = (T)c.weights[i];
    for (int a = 0; a < 3; ++a) {
      e.n[a] = (T)n[a];
      e.delta[a] = (T)delta[a];
      e.s[a] = s[a];
    }
    e.scale = (T)c.scales[i];
    e.inv_scale = (T)(1.0 / c.scales[i]);
    e.plane = i;
    e.plane_el = (int64_t)i * ncell;
    e.plane_off = (int64_t)i * ncell * esize;
    e.invw = e.w != T(0) ? T(1) / e.w : T(0);
    e.psel = s[0] > 0 ? 0x05040302u : 0x01000706u;
    e.rnd = plane_random(i);
  }
  // each slot carries its wave's sum of n_i w_i (the stored values, in FP64)
  const int m = c.nb / waves_for(c.nb);
  for (int q = 0; q < c.nb / m; ++q) {
    double nw[3] = {0.0, 0.0, 0.0};
    for (int k = q * m; k < (q + 1) * m; ++k)
      for (int a = 0; a < 3; ++a) nw[a] += (double)tab[k].n[a] * (double)tab[k].w;
    for (int k = q * m; k < (q + 1) * m; ++k)
      for (int a = 0; a < 3; ++a) tab[k].nwq[a] = nw[a];
  }
}

// The pair kernel's compact slot records, from the FP32 direction table.
void build_pair_tables(const std::vector<DirTab<float>> &tab, std::vector<PairTab> &pt,
                       std::vector<PairColl> &pc) {
  pt.assign(tab.size(), PairTab{});
  pc.assign(tab.size(), PairColl{});
  for (size_t k = 0; k < tab.size(); ++k) {
    const DirTab<float> &e = tab[k];
    PairTab &a = pt[k];
    a.wx0 = e.wx[0];
    a.wx1 = e.wx[1];
    a.wy0 = e.wy[0];
    a.wy1 = e.wy[1];
    a.wz_new = e.wz_new;
    a.wz_old = e.wz_old;
    a.w = e.w;
    a.invw = e.invw;
    a.n0 = e.n[0];
    a.n1 = e.n[1];
    a.n2 = e.n[2];
    a.scale = e.scale;
    a.plane_off = e.plane_off;
    a.row_off = (int32_t)e.row_off;
    a.flags = (e.s[0] > 0 ? kPairSxPos : 0u) | (e.dzn ? kPairDzn : 0u) |
              (e.active ? kPairActive : 0u);
    PairColl &b = pc[k];
    b.w = e.w;
    b.n0 = e.n[0];
    b.n1 = e.n[1];
    b.n2 = e.n[2];
    b.inv_scale = e.active ? e.inv_scale : 0.0f;   // 0 marks a padding slot
    b.rnd = e.rnd;
    b.plane_off = e.plane_off;
  }
}

// True when every wave's sum of n_i w_i is exactly 0 (a centrally symmetric
// rule whose antipodal pairs never straddle two waves): the kernels' FP64
// reference term of the flux is then exactly 0 and is skipped (unless
// LBRT_FP64_FLUX_TERM is set, which keeps it: the same bits, for checking).
template <typename T>
bool all_nwq_zero(const std::vector<DirTab<T>> &tab) {
  for (const DirTab<T> &e : tab)
    for (int a = 0; a < 3; ++a)
      if (e.nwq[a] != 0.0) return false;
  return true;
}

int ensure_partials(lbrt_ctx *c, int nblocks) {
  if (nblocks <= c->partials_cap) return LBRT_OK;
  if (c->partials) (void)hipFree(c->partials);
  c->partials = nullptr;
  c->partials_cap = 0;
  hipError_t e = hipMalloc(&c->partials, sizeof(double) * kStepPartials * (size_t)nblocks);
  if (e != hipSuccess) return fail(LBRT_E_NOMEM, "hipMalloc(diagnostic partials): %s",
                                   hipGetErrorString(e));
  c->partials_cap = nblocks;
  return LBRT_OK;
}

// Kernel parameters of the context for tile plan `mode` (variant 0).
KParams make_params(const lbrt_ctx *c, int mode) {
  const lbrt_desc &d = c->desc;
  KParams p{};
  p.nx = d.nx;
  p.ny = d.ny;
  p.nz = d.nz;
  p.ndir = d.ndir;
  p.ncell = (int64_t)d.nx * d.ny * d.nz;
  p.tx = c->tile.tx;
  p.ty = c->tile.ty;
  p.txlog = 0;
  while ((1 << p.txlog) < p.tx) ++p.txlog;
  p.zlen = c->zlen;
  p.nty = (d.ny + p.ty - 1) / p.ty;
  p.main_ty0 = 1;
  if (mode == 1) {
    p.pair = 1;
    p.pair_x0 = pair_face_columns(d) ? kPairX0 : 0;
    p.pair_xend = d.nx - p.pair_x0;
    p.pair_tab = c->pair_tab_dev;
    p.pair_coll = c->pair_coll_dev;
    p.ntx = pair_ntx(d.nx);
    p.main_nty = d.ny - 2;
  } else {
    // main kernel: every x tile (a ragged last tile masks its extra lanes), y
    // tiles whose halo rows are inside the box
    p.ntx = (d.nx + p.tx - 1) / p.tx;
    p.main_nty = std::max(0, (d.ny - 1 - p.ty) / p.ty);
  }
  const lbrt_ctx::Plan &pl = c->plan[mode][0];
  p.main_zr0 = pl.zr0;
  p.main_nzr = pl.nzr;
  p.nblocks = p.ntx * p.main_nty * p.main_nzr;
  p.ngeneral = (int)pl.general.size();
  p.general_list = pl.dev;
  for (int a = 0; a < 3; ++a) p.periodic[a] = d.bc[2 * a] == LBRT_BC_PERIODIC;
  p.mode = d.collision;
  p.lambda_iters = d.lambda_iters;
  p.flags = 0;
  if (c->paired) p.flags |= KF_PAIRED;
  if (d.moving_fluid) p.flags |= KF_MOVING;
  if (d.lambda_aniso == 0.0) p.flags |= KF_LAMZERO;
  if (c->nwq_zero) p.flags |= KF_NWQZERO;
  if (is_reduced(d.storage) && d.rounding == LBRT_ROUND_STOCHASTIC) p.flags |= KF_STOCH;
  p.e_off = e_offset(d.storage, d.ndir, p.ncell);
  p.dt = d.dt;  // time step in length units (c = 1)
  p.lam = d.lambda_aniso;
  return p;
}

KParams make_params(const lbrt_ctx *c) { return make_params(c, c->pair ? 1 : 0); }

// The same with the tile plan variant for inflow ghost planes on a z face.
void use_zinflow_variant(const lbrt_ctx *c, KParams &p) {
  const lbrt_ctx::Plan &pl = c->plan[p.pair ? 1 : 0][1];
  p.main_zr0 = pl.zr0;
  p.main_nzr = pl.nzr;
  p.nblocks = p.ntx * p.main_nty * p.main_nzr;
  p.ngeneral = (int)pl.general.size();
  p.general_list = pl.dev;
}

// Splits the cells between the main (mode 0) or pair (mode 1) kernel and the
// general kernel, which takes everything else in z ranges of zlen_general
// planes.  Mode 0: main tiles are the context's xy tiles of the interior rows
// (every x); mode 1: pair tiles cover x in [2, nx - 2) of rows [1, ny - 1),
// and the general kernel takes the columns x < 2 and x >= nx - 2 (2 x 32
// tiles) and the rows 0 and ny - 1.  With zlo_inflow / zhi_inflow, the first
// / last z range (next to a z face with inflow ghost planes) of the interior
// goes to the general kernel too.
int plan_tiles(lbrt_ctx *c, int mode, int variant, bool zlo_inflow, bool zhi_inflow) {
  const lbrt_desc &d = c->desc;
  const int tx = c->tile.tx, ty = c->tile.ty;
  int txlog = 0;
  while ((1 << txlog) < tx) ++txlog;
  const int nzr = (d.nz + c->zlen - 1) / c->zlen;
  int zr0 = zlo_inflow ? 1 : 0;
  int zr1 = nzr - (zhi_inflow ? 1 : 0);
  const bool rows = mode == 1 ? d.ny > 2 : std::max(0, (d.ny - 1 - ty) / ty) > 0;
  if (zr1 < zr0 || !rows) zr1 = zr0;
  lbrt_ctx::Plan &pl = c->plan[mode][variant];
  pl.zr0 = zr0;
  pl.nzr = zr1 - zr0;
  const bool any_main = zr1 > zr0;
  const int zm0 = std::min(d.nz, zr0 * c->zlen), zm1 = std::min(d.nz, zr1 * c->zlen);
  std::vector<GenTile> list;
  auto add = [&](int x0, int y0, int xe, int ye, int tl, int z0, int z1) {
    for (int zb = z0; zb < z1; zb += c->zlen_general) {
      GenTile g{};
      g.x0 = x0;
      g.y0 = y0;
      g.zb = zb;
      g.ze = std::min(z1, zb + c->zlen_general);
      g.xe = xe;
      g.ye = ye;
      g.txlog = tl;
      list.push_back(g);
    }
  };
  if (mode == 0) {
    const int ntx_all = (d.nx + tx - 1) / tx;
    const int nty = (d.ny + ty - 1) / ty;
    const int main_nty = std::max(0, (d.ny - 1 - ty) / ty);
    for (int tiy = 0; tiy < nty; ++tiy) {
      for (int tix = 0; tix < ntx_all; ++tix) {
        const bool main_xy = any_main && tiy >= 1 && tiy <= main_nty;
        if (!main_xy) {
          add(tix * tx, tiy * ty, d.nx, d.ny, txlog, 0, d.nz);
        } else {
          add(tix * tx, tiy * ty, d.nx, d.ny, txlog, 0, zm0);
          add(tix * tx, tiy * ty, d.nx, d.ny, txlog, zm1, d.nz);
        }
      }
    }
  } else {
    const int xa = pair_face_columns(d) ? kPairX0 : 0, xb = d.nx - xa;
    // the face columns of a periodic x axis, every row
    if (xa > 0)
      for (int x0 : {0, xb})
        for (int y0 = 0; y0 < d.ny; y0 += 32) add(x0, y0, x0 + kPairX0, d.ny, 1, 0, d.nz);
    // rows 0 and ny - 1 between them, and the interior rows' z ranges that
    // the pair kernel does not march
    for (int y = 0; y < d.ny; ++y) {
      const bool face_row = y == 0 || y == d.ny - 1;
      for (int x0 = xa; x0 < xb; x0 += 64) {
        if (face_row || !any_main) {
          add(x0, y, xb, y + 1, 6, 0, d.nz);
        } else {
          add(x0, y, xb, y + 1, 6, 0, zm0);
          add(x0, y, xb, y + 1, 6, zm1, d.nz);
        }
      }
    }
  }
  pl.general = list;
  if (pl.dev) (void)hipFree(pl.dev);
  pl.dev = nullptr;
  if (list.empty()) return LBRT_OK;
  hipError_t e = hipMalloc(&pl.dev, sizeof(GenTile) * list.size());
  if (e == hipSuccess)
    e = hipMemcpy(pl.dev, list.data(), sizeof(GenTile) * list.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(LBRT_E_NOMEM, "tile list: %s", hipGetErrorString(e));
  return LBRT_OK;
}

// Both modes' plans, both variants (mode 1 only where the pair kernel runs).
int plan_all(lbrt_ctx *c) {
  const lbrt_desc &d = c->desc;
  const bool zlo = d.bc[LBRT_FACE_MZ] == LBRT_BC_INFLOW, zhi = d.bc[LBRT_FACE_PZ] == LBRT_BC_INFLOW;
  for (int mode = 0; mode < (c->pair ? 2 : 1); ++mode) {
    int rc = plan_tiles(c, mode, 0, false, false);
    if (rc == LBRT_OK) rc = plan_tiles(c, mode, 1, zlo, zhi);
    if (rc != LBRT_OK) return rc;
  }
  return LBRT_OK;
}

// Checks the inflow planes of a call and fills the compact per-slot ghost
// table (which inflow_table_kernel expands into InflowArgs on the device).
int build_inflow(const lbrt_ctx *c, const lbrt_inflow *inflow, int32_t ninflow,
                 InflowCompact &in, bool &xghosts, bool &zghosts) {
  const lbrt_desc &d = c->desc;
  if (ninflow < 0 || ninflow > LBRT_MAX_INFLOW)
    return fail(LBRT_E_INVAL, "ninflow = %d outside [0, %d]", ninflow, (int)LBRT_MAX_INFLOW);
  if (ninflow > 0 && !inflow) return fail(LBRT_E_INVAL, "inflow is NULL but ninflow > 0");
  std::memset(&in, 0, sizeof(in));
  in.n = ninflow;
  for (int j = 0; j < ninflow; ++j) {
    const lbrt_inflow &pl = inflow[j];
    if (pl.face < 0 || pl.face > 5) return fail(LBRT_E_INVAL, "inflow[%d].face = %d", j, pl.face);
    if (d.bc[pl.face] != LBRT_BC_INFLOW)
      return fail(LBRT_E_INVAL, "inflow[%d]: face %d is not an inflow face", j, pl.face);
    if (pl.dir < 0 || pl.dir >= d.ndir) return fail(LBRT_E_INVAL, "inflow[%d].dir = %d", j, pl.dir);
    if (!pl.values) return fail(LBRT_E_INVAL, "inflow[%d].values is NULL", j);
    const int axis = pl.face >> 1;
    const double comp = c->dirs[3 * pl.dir + axis];
    const bool enters = (pl.face & 1) == 0 ? comp > 0.0 : comp < 0.0;
    if (!enters)
      return fail(LBRT_E_INVAL, "inflow[%d]: direction %d does not enter through face %d", j,
                  pl.dir, pl.face);
    for (int k = 0; k < j; ++k)
      if (in.face[k] == pl.face && in.dir[k] == pl.dir)
        return fail(LBRT_E_INVAL, "inflow[%d]: (face %d, dir %d) listed twice", j, pl.face,
                    pl.dir);
    in.face[j] = pl.face;
    in.dir[j] = pl.dir;
    in.ptr[j] = pl.values;
  }
  // per processing slot and axis: the ghost plane that slot pulls from
  for (int k = 0; k < LBRT_MAX_DIRS; ++k)
    for (int a = 0; a < 3; ++a) in.slot_plane[k][a] = -1;
  xghosts = zghosts = false;
  for (int j = 0; j < ninflow; ++j) {
    xghosts |= (in.face[j] >> 1) == 0;
    zghosts |= (in.face[j] >> 1) == 2;
  }
  for (int k = 0; k < d.ndir; ++k) {
    const int i = c->order[k];
    for (int a = 0; a < 3; ++a) {
      const double comp = c->dirs[3 * i + a];
      if (comp == 0.0) continue;
      const int face = 2 * a + (comp > 0.0 ? 0 : 1);
      for (int j = 0; j < ninflow; ++j)
        if (in.face[j] == face && in.dir[j] == i) in.slot_plane[k][a] = (int8_t)j;
    }
  }
  return LBRT_OK;
}

int total_partials(const KParams &p) { return p.nblocks + p.ngeneral + zface_blocks(p); }

// What a step call needs after its arguments are checked: the kernel
// parameters (tile plan for the call's ghost planes) and the compact ghost
// table.
struct StepCall {
  KParams p;
  InflowCompact in;
  StepLauncher launch;
};

int prepare_step(lbrt_ctx *c, void *I_a, void *I_b, const float *kappa_a, const float *kappa_s,
                 const float *eta, const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
                 int32_t nsteps, StepCall &call) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (nsteps < 0) return fail(LBRT_E_INVAL, "nsteps = %d < 0", nsteps);
  if (!I_a || !I_b) return fail(LBRT_E_INVAL, "population buffers are required");
  if (I_a == I_b) return fail(LBRT_E_INVAL, "I_a and I_b must be distinct (ping-pong)");
  const lbrt_desc &d = c->desc;
  const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
  const size_t bytes = (size_t)state_bytes(d.storage, d.ndir, ncell);
  const char *a = static_cast<const char *>(I_a), *b = static_cast<const char *>(I_b);
  if (a < b + bytes && b < a + bytes) return fail(LBRT_E_INVAL, "I_a and I_b overlap");
  if (!kappa_a || !kappa_s || !eta) return fail(LBRT_E_INVAL, "kappa_a, kappa_s, eta required");
  if (d.moving_fluid && !vel) return fail(LBRT_E_INVAL, "moving fluid: vel is required");
  if (!d.moving_fluid && vel) return fail(LBRT_E_INVAL, "vel given but moving_fluid is off");
  bool xghosts, zghosts;
  int rc = build_inflow(c, inflow, ninflow, call.in, xghosts, zghosts);
  if (rc != LBRT_OK) return rc;
  KParams &p = call.p;
  p = make_params(c);
  if (xghosts) p.flags |= KF_XGHOSTS;
  // z ranges next to an inflow z face go to the general kernel
  if (zghosts) use_zinflow_variant(c, p);
  call.launch = step_launcher(d.storage, c->bucket, d.moving_fluid != 0);
  if (!call.launch)
    return fail(LBRT_E_UNSUPPORTED, "no kernel for storage %d, %d directions", d.storage,
                d.ndir);
  return LBRT_OK;
}

int moments_impl(lbrt_ctx *c, const void *I, void *E, void *F, hipStream_t s);

// The launches of a step call: the ghost table (when the context has an
// inflow face, or always with `table_always`), the diagnostics clear, then
// per step the z-face fluxes, the step kernels and the diagnostics
// reduction.  `partials` holds total_partials(p) rows when diag is given.
int run_steps(lbrt_ctx *c, const StepCall &call, void *I_a, void *I_b, const float *kappa_a,
              const float *kappa_s, const float *eta, const float *vel, int32_t nsteps, void *E,
              void *F, double *diag, double *partials, InflowArgs *table, bool table_always,
              hipStream_t s) {
  const lbrt_desc &d = c->desc;
  const KParams &p = call.p;
  hipError_t e;
  if (table_always || c->any_inflow_face) {
    e = launch_inflow_table(call.in, table, s);
    if (e != hipSuccess) return hip_fail(e, "lbrt_step: writing the inflow table");
  }
  if (diag) {
    e = launch_fill_f64(diag, kDiag, 0.0, s);
    if (e != hipSuccess) return hip_fail(e, "lbrt_step: clearing diag");
  }
  if (nsteps == 0) {
    if (E || F) return moments_impl(c, I_a, E, F, s);
    return LBRT_OK;
  }
  const int nparts = total_partials(p);
  for (int k = 0; k < nsteps; ++k) {
    const void *src = (k & 1) ? I_b : I_a;
    void *dst = (k & 1) ? I_a : I_b;
    KParams pk = p;
    // this step's stochastic rounding seed (one per step of the context)
    pk.seed = (uint32_t)splitmix64(0x5eedull ^ (c->round_seq++ * 0x9e3779b97f4a7c15ull));
    const bool last = k == nsteps - 1;
    if (diag) {
      pk.flags |= KF_DIAG;
      e = launch_zface(d.storage, src, c->tab_dev, p, table,
                       partials + (size_t)(p.nblocks + p.ngeneral) * kStepPartials, s);
      if (e != hipSuccess) return hip_fail(e, "lbrt_step: launching the z-face flux kernel");
    }
    if (last && (E || F)) pk.flags |= KF_WRITE_EF;
    e = call.launch(src, dst, kappa_a, kappa_s, eta, vel, c->tab_dev, pk, table,
                    last ? E : nullptr, last ? F : nullptr, partials, s);
    if (e != hipSuccess) return hip_fail(e, "lbrt_step: launching the step kernel");
    if (diag) {
      e = launch_diag_reduce(partials, nparts, diag, k == 0, s);
      if (e != hipSuccess) return hip_fail(e, "lbrt_step: reducing diagnostics");
    }
  }
  return LBRT_OK;
}

int moments_impl(lbrt_ctx *c, const void *I, void *E, void *F, hipStream_t s) {
  if (!E && !F) return LBRT_OK;
  KParams p = make_params(c);
  hipError_t e = launch_moments(c->desc.storage, I, c->tab_dev, p, E, F, s);
  if (e != hipSuccess) return hip_fail(e, "lbrt_moments");
  return LBRT_OK;
}
}  // namespace

extern "C" {

const char *lbrt_last_error(void) { return g_err.c_str(); }

int lbrt_validate(const lbrt_desc *d) {
  if (!d) return fail(LBRT_E_INVAL, "desc is NULL");
  if (d->nx < 2 || d->ny < 2 || d->nz < 2)
    return fail(LBRT_E_INVAL, "grid %d x %d x %d: every dimension must be >= 2", d->nx, d->ny,
                d->nz);
  const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
  if (ncell >= (int64_t)1 << 31 || (int64_t)d->nx * d->ny >= (int64_t)1 << 28)
    return fail(LBRT_E_INVAL, "grid too large: nx*ny*nz must be < 2^31 and nx*ny < 2^28");
  if (!(d->dx > 0.0) || !std::isfinite(d->dx)) return fail(LBRT_E_INVAL, "dx must be > 0");
  if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(LBRT_E_CFL, "dt must be > 0");
  if (d->dt > d->dx)
    return fail(LBRT_E_CFL, "dt = %g > dx = %g: the trilinear pull spans one cell only",
                d->dt, d->dx);
  if (d->ndir < 2 || d->ndir > LBRT_MAX_DIRS)
    return fail(LBRT_E_INVAL, "ndir = %d outside [2, %d]", d->ndir, (int)LBRT_MAX_DIRS);
  if (!d->dirs || !d->weights) return fail(LBRT_E_INVAL, "dirs and weights are required");
  for (int f = 0; f < 6; ++f)
    if (d->bc[f] < LBRT_BC_OUTFLOW || d->bc[f] > LBRT_BC_INFLOW)
      return fail(LBRT_E_INVAL, "bc[%d] = %d is not a boundary kind", f, d->bc[f]);
  if (!is_periodic_pair_ok(d->bc))
    return fail(LBRT_E_INVAL, "periodic boundaries must be set on both faces of an axis");
  if (d->storage < LBRT_FP32 || d->storage > LBRT_FP16_SHIFTED)
    return fail(LBRT_E_INVAL, "storage = %d is not a storage type", d->storage);
  if (d->collision < LBRT_COLL_IMPLICIT || d->collision > LBRT_COLL_LAMBDA)
    return fail(LBRT_E_INVAL, "collision = %d is not a collision kind", d->collision);
  if (d->rounding != LBRT_ROUND_STOCHASTIC && d->rounding != LBRT_ROUND_NEAREST)
    return fail(LBRT_E_INVAL, "rounding = %d is not a rounding mode", d->rounding);
  if (d->collision == LBRT_COLL_LAMBDA && d->lambda_iters < 1)
    return fail(LBRT_E_INVAL, "lambda_iters must be >= 1");
  if (!std::isfinite(d->lambda_aniso)) return fail(LBRT_E_INVAL, "lambda_aniso not finite");
  if (d->moving_fluid) {
    if (d->collision != LBRT_COLL_IMPLICIT)
      return fail(LBRT_E_UNSUPPORTED, "moving fluid needs the implicit collision");
    if (d->lambda_aniso != 0.0)
      return fail(LBRT_E_UNSUPPORTED, "moving fluid supports isotropic scattering only");
  }
  double s0 = 0.0, s1[3] = {0, 0, 0}, s2[3][3] = {{0}};
  for (int i = 0; i < d->ndir; ++i) {
    const double *n = d->dirs + 3 * i;
    const double w = d->weights[i];
    if (!std::isfinite(w) || w == 0.0)
      return fail(LBRT_E_QUAD, "weight %d = %g must be finite and nonzero", i, w);
    const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (!(std::fabs(len - 1.0) <= 1e-12))
      return fail(LBRT_E_QUAD, "direction %d has length %.17g, not 1", i, len);
    s0 += w;
    for (int a = 0; a < 3; ++a) {
      s1[a] += w * n[a];
      for (int b = 0; b < 3; ++b) s2[a][b] += w * n[a] * n[b];
    }
    if (d->scale && !(d->scale[i] > 0.0 && std::isfinite(d->scale[i])))
      return fail(LBRT_E_INVAL, "scale %d = %g must be > 0", i, d->scale[i]);
  }
  if (std::fabs(s0 - 1.0) > 1e-12) return fail(LBRT_E_QUAD, "sum w = %.17g, not 1", s0);
  for (int a = 0; a < 3; ++a) {
    if (std::fabs(s1[a]) > 1e-12) return fail(LBRT_E_QUAD, "sum w n[%d] = %.3g, not 0", a, s1[a]);
    for (int b = 0; b < 3; ++b) {
      const double want = a == b ? 1.0 / 3.0 : 0.0;
      if (std::fabs(s2[a][b] - want) > 1e-12)
        return fail(LBRT_E_QUAD, "sum w n n[%d][%d] = %.17g, not %.17g", a, b, s2[a][b], want);
    }
  }
  return LBRT_OK;
}

int lbrt_init(const lbrt_desc *d, lbrt_ctx **out) {
  if (!out) return fail(LBRT_E_INVAL, "out is NULL");
  int rc = lbrt_validate(d);
  if (rc != LBRT_OK) return rc;
  lbrt_ctx *c = new lbrt_ctx();
  c->desc = *d;
  c->desc.dirs = c->desc.weights = c->desc.scale = nullptr;
  c->dirs.assign(d->dirs, d->dirs + 3 * d->ndir);
  c->weights.assign(d->weights, d->weights + d->ndir);
  c->scales.resize(d->ndir);
  const bool reduced = is_reduced(d->storage);
  for (int i = 0; i < d->ndir; ++i)
    c->scales[i] = reduced ? (d->scale ? d->scale[i] : std::fabs(d->weights[i])) : 1.0;
  c->bucket = bucket_for(d->ndir);
  c->nb = kBuckets[c->bucket];
  if (!step_launcher(d->storage, c->bucket, d->moving_fluid != 0)) {
    rc = fail(LBRT_E_UNSUPPORTED,
              "no compiled kernel for storage %d with %d directions (%s fluid)", d->storage,
              d->ndir, d->moving_fluid ? "moving" : "static");
    delete c;
    return rc;
  }
  // Antipodal pairing (every n_i has a partner -n_i) puts each pair in
  // adjacent processing slots.
  std::vector<int> partner(d->ndir, -1);
  bool paired = (d->ndir % 2) == 0;
  for (int i = 0; i < d->ndir && paired; ++i) {
    for (int j = 0; j < d->ndir; ++j) {
      if (j == i) continue;
      const double *a = &c->dirs[3 * i], *b = &c->dirs[3 * j];
      if (std::fabs(a[0] + b[0]) < 1e-12 && std::fabs(a[1] + b[1]) < 1e-12 &&
          std::fabs(a[2] + b[2]) < 1e-12) {
        partner[i] = j;
        break;
      }
    }
    if (partner[i] < 0) paired = false;
  }
  c->order.clear();
  if (paired) {
    std::vector<bool> used(d->ndir, false);
    for (int i = 0; i < d->ndir; ++i) {
      if (used[i]) continue;
      const int j = partner[i];
      if (used[j] || partner[j] != i) { paired = false; break; }
      c->order.push_back(i);
      c->order.push_back(j);
      used[i] = used[j] = true;
    }
  }
  if (!paired) {
    c->order.resize(d->ndir);
    for (int i = 0; i < d->ndir; ++i) c->order[i] = i;
  }
  c->paired = paired;
  c->tile = default_tile(d->nx, d->ny, d->nz);
  if (const char *env = std::getenv("LBRT_ZLEN_GENERAL")) {
    const int v = std::atoi(env);
    if (v > 0) c->zlen_general = v;
  }
  (void)hipGetDevice(&c->device);
  if (c->device < 0 || c->device >= kMaxDevices) {
    rc = fail(LBRT_E_UNSUPPORTED, "device %d: at most %d devices", c->device, kMaxDevices);
    delete c;
    return rc;
  }
  {
    // once per device, with that device current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
      void *ptr = nullptr;
      const hipError_t es = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (es != hipSuccess || !ptr) {
        rc = fail(LBRT_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(es));
        delete c;
        return rc;
      }
      g_scratch_ptr[c->device] = ptr;
    }
    c->scratch = static_cast<unsigned char *>(g_scratch_ptr[c->device]);
  }

  hipError_t e;
  size_t tab_bytes;
  if (d->storage == LBRT_FP64) {
    std::vector<DirTab<double>> tab;
    build_table(*c, tab);
    c->nwq_zero = all_nwq_zero(tab) && !std::getenv("LBRT_FP64_FLUX_TERM");
    tab_bytes = sizeof(DirTab<double>) * tab.size();
    c->tab_bytes = tab_bytes;
    e = hipMalloc(&c->tab_dev, tab_bytes);
    if (e == hipSuccess) e = hipMemcpy(c->tab_dev, tab.data(), tab_bytes, hipMemcpyHostToDevice);
  } else {
    std::vector<DirTab<float>> tab;
    build_table(*c, tab);
    c->nwq_zero = all_nwq_zero(tab) && !std::getenv("LBRT_FP64_FLUX_TERM");
    tab_bytes = sizeof(DirTab<float>) * tab.size();
    c->tab_bytes = tab_bytes;
    e = hipMalloc(&c->tab_dev, tab_bytes);
    if (e == hipSuccess) e = hipMemcpy(c->tab_dev, tab.data(), tab_bytes, hipMemcpyHostToDevice);
    std::vector<PairTab> pt;
    std::vector<PairColl> pcl;
    build_pair_tables(tab, pt, pcl);
    if (e == hipSuccess) e = hipMalloc(&c->pair_tab_dev, sizeof(PairTab) * pt.size());
    if (e == hipSuccess)
      e = hipMemcpy(c->pair_tab_dev, pt.data(), sizeof(PairTab) * pt.size(),
                    hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&c->pair_coll_dev, sizeof(PairColl) * pcl.size());
    if (e == hipSuccess)
      e = hipMemcpy(c->pair_coll_dev, pcl.data(), sizeof(PairColl) * pcl.size(),
                    hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMalloc(&c->scales_dev, sizeof(double) * d->ndir);
  if (e == hipSuccess)
    e = hipMemcpy(c->scales_dev, c->scales.data(), sizeof(double) * d->ndir,
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->weights_dev, sizeof(double) * d->ndir);
  if (e == hipSuccess)
    e = hipMemcpy(c->weights_dev, c->weights.data(), sizeof(double) * d->ndir,
                  hipMemcpyHostToDevice);
  {
    std::vector<CoupDir> cd(d->ndir);
    for (int i = 0; i < d->ndir; ++i) {
      const double *n = &c->dirs[3 * i];
      cd[i] = CoupDir{{n[0], n[1], n[2]},
                      {n[0] * n[0], n[0] * n[1], n[0] * n[2], n[1] * n[1], n[1] * n[2], n[2] * n[2]},
                      c->scales[i], c->weights[i]};
    }
    if (e == hipSuccess) e = hipMalloc(&c->coup_dev, sizeof(CoupDir) * d->ndir);
    if (e == hipSuccess)
      e = hipMemcpy(c->coup_dev, cd.data(), sizeof(CoupDir) * d->ndir, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    rc = fail(e == hipErrorOutOfMemory ? LBRT_E_NOMEM : LBRT_E_HIP, "lbrt_init: %s",
              hipGetErrorString(e));
    lbrt_destroy(c);
    return rc;
  }
  // The pair kernel (two x cells per lane) runs the interior where it is
  // compiled, on grids with even nx, for rules whose flux sums need no FP64
  // reference term; LBRT_PAIR=0 keeps the main kernel (speed only).
  {
    const char *env = std::getenv("LBRT_PAIR");
    c->pair = pair_available(d->storage, c->nb, d->moving_fluid != 0) && d->nx % 2 == 0 &&
              d->nx >= 8 && d->ny >= 3 && c->nwq_zero && !(env && std::strcmp(env, "0") == 0);
  }
  {
    const int64_t xy = c->pair ? (int64_t)pair_ntx(d->nx) * (d->ny - 2)
                               : (int64_t)((d->nx + c->tile.tx - 1) / c->tile.tx) *
                                     ((d->ny + c->tile.ty - 1) / c->tile.ty);
    c->zlen = default_zlen(d->nz, xy, c->pair ? 4096 : 8192);
  }
  rc = plan_all(c);
  if (rc != LBRT_OK) {
    lbrt_destroy(c);
    return rc;
  }
  KParams p = make_params(c);
  rc = ensure_partials(c, total_partials(p));
  if (rc == LBRT_OK) {
    // the ghost table starts empty; calls on a context with an inflow face
    // rewrite it on their stream
    InflowArgs none;
    std::memset(&none, 0, sizeof(none));
    e = hipMalloc(&c->inflow_dev, sizeof(InflowArgs));
    if (e == hipSuccess)
      e = hipMemcpy(c->inflow_dev, &none, sizeof(InflowArgs), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = fail(LBRT_E_NOMEM, "context buffers: %s", hipGetErrorString(e));
  }
  for (int f = 0; f < 6; ++f) c->any_inflow_face |= d->bc[f] == LBRT_BC_INFLOW;
  if (rc != LBRT_OK) {
    lbrt_destroy(c);
    return rc;
  }
  *out = c;
  return LBRT_OK;
}

void lbrt_destroy(lbrt_ctx *c) {
  if (!c) return;
  if (c->tab_dev) (void)hipFree(c->tab_dev);
  if (c->pair_tab_dev) (void)hipFree(c->pair_tab_dev);
  if (c->pair_coll_dev) (void)hipFree(c->pair_coll_dev);
  if (c->scales_dev) (void)hipFree(c->scales_dev);
  if (c->weights_dev) (void)hipFree(c->weights_dev);
  if (c->coup_dev) (void)hipFree(c->coup_dev);
  if (c->partials) (void)hipFree(c->partials);
  if (c->inflow_dev) (void)hipFree(c->inflow_dev);
  for (auto &m : c->plan)
    for (auto &pl : m)
      if (pl.dev) (void)hipFree(pl.dev);
  if (c->adj_work) (void)hipFree(c->adj_work);
  delete c;
}

int lbrt_step(lbrt_ctx *c, void *I_a, void *I_b, const float *kappa_a, const float *kappa_s,
              const float *eta, const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
              int32_t nsteps, void *E, void *F, double *diag, void *stream) {
  StepCall call;
  int rc = prepare_step(c, I_a, I_b, kappa_a, kappa_s, eta, vel, inflow, ninflow, nsteps, call);
  if (rc != LBRT_OK) return rc;
  if (diag) {
    rc = ensure_partials(c, total_partials(call.p));
    if (rc != LBRT_OK) return rc;
  }
  return run_steps(c, call, I_a, I_b, kappa_a, kappa_s, eta, vel, nsteps, E, F, diag,
                   c->partials, c->inflow_dev, c->any_inflow_face,
                   static_cast<hipStream_t>(stream));
}

int lbrt_step_noalloc(lbrt_ctx *c, void *I_a, void *I_b, const float *kappa_a,
                      const float *kappa_s, const float *eta, const float *vel,
                      const lbrt_inflow *inflow, int32_t ninflow, int32_t nsteps, void *E,
                      void *F, double *diag, void *stream) {
  StepCall call;
  int rc = prepare_step(c, I_a, I_b, kappa_a, kappa_s, eta, vel, inflow, ninflow, nsteps, call);
  if (rc != LBRT_OK) return rc;
  if (!c->scratch) return fail(LBRT_E_HIP, "lbrt_step_noalloc: no scratch on device %d", c->device);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != c->device)
    return fail(LBRT_E_INVAL, "lbrt_step_noalloc: the context's device %d is not current (%d)",
                c->device, cur);
  const int need = total_partials(call.p);
  if (diag && need > kScratchMaxPartials)
    return fail(LBRT_E_INVAL,
                "lbrt_step_noalloc: diagnostics need %d block partials (%zu bytes), more than "
                "the %d (%zu bytes) of the fixed scratch; use lbrt_step or pass diag = NULL",
                need, (size_t)need * sizeof(double) * kStepPartials, kScratchMaxPartials,
                kScratchBytes - kScratchTableBytes);
  InflowArgs *table = reinterpret_cast<InflowArgs *>(c->scratch);
  double *partials = reinterpret_cast<double *>(c->scratch + kScratchTableBytes);
  return run_steps(c, call, I_a, I_b, kappa_a, kappa_s, eta, vel, nsteps, E, F, diag, partials,
                   table, true, static_cast<hipStream_t>(stream));
}

int lbrt_adjoint_step(lbrt_ctx *c, const void *I_n, const void *lam_next, void *lam_out,
                      int32_t detector_face, void *g_kappa_a, void *g_kappa_s, void *g_eta,
                      const float *kappa_a, const float *kappa_s, const float *eta,
                      const float *vel, const lbrt_inflow *inflow, int32_t ninflow,
                      void *stream) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  const lbrt_desc &d = c->desc;
  if (d.storage != LBRT_FP32 && d.storage != LBRT_FP64)
    return fail(LBRT_E_UNSUPPORTED, "the adjoint needs FP32 or FP64 storage");
  if (d.collision != LBRT_COLL_IMPLICIT || d.lambda_aniso != 0.0)
    return fail(LBRT_E_UNSUPPORTED, "the adjoint covers the implicit collision with lambda = 0");
  if (!I_n || !lam_next || !lam_out) return fail(LBRT_E_INVAL, "I_n, lam_next, lam_out required");
  if (!g_kappa_a || !g_kappa_s || !g_eta) return fail(LBRT_E_INVAL, "gradients required");
  if (!kappa_a || !kappa_s || !eta) return fail(LBRT_E_INVAL, "kappa_a, kappa_s, eta required");
  if (d.moving_fluid && !vel) return fail(LBRT_E_INVAL, "moving fluid: vel is required");
  if (!d.moving_fluid && vel) return fail(LBRT_E_INVAL, "vel given but moving_fluid is off");
  if (detector_face < -1 || detector_face > 5)
    return fail(LBRT_E_INVAL, "detector_face = %d outside [-1, 5]", detector_face);
  const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
  const size_t bytes = storage_bytes(d.storage) * (size_t)ncell * d.ndir;
  const char *ln = static_cast<const char *>(lam_next), *lo = static_cast<const char *>(lam_out);
  if (ln < lo + bytes && lo < ln + bytes) return fail(LBRT_E_INVAL, "lam_next and lam_out overlap");
  InflowCompact in;
  bool xghosts, zghosts;
  int rc = build_inflow(c, inflow, ninflow, in, xghosts, zghosts);
  if (rc != LBRT_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!c->adj_work) {
    hipError_t e = hipMalloc(&c->adj_work, bytes);
    if (e != hipSuccess) {
      c->adj_work = nullptr;
      return fail(LBRT_E_NOMEM, "hipMalloc(adjoint work buffer, %zu bytes): %s", bytes,
                  hipGetErrorString(e));
    }
  }
  if (c->any_inflow_face) {
    const hipError_t e0 = launch_inflow_table(in, c->inflow_dev, s);
    if (e0 != hipSuccess) return hip_fail(e0, "lbrt_adjoint_step: writing the inflow table");
  }
  KParams p = make_params(c);
  hipError_t e = launch_adjoint(d.storage, I_n, lam_next, lam_out, c->adj_work, detector_face,
                                g_kappa_a, g_kappa_s, g_eta, kappa_a, kappa_s, eta, vel,
                                c->tab_dev, p, c->inflow_dev, s);
  if (e != hipSuccess) return hip_fail(e, "lbrt_adjoint_step");
  return LBRT_OK;
}

int lbrt_moments(lbrt_ctx *c, const void *I, void *E, void *F, void *stream) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (!I) return fail(LBRT_E_INVAL, "I is NULL");
  return moments_impl(c, I, E, F, static_cast<hipStream_t>(stream));
}

int lbrt_coupling(lbrt_ctx *c, const void *I, const float *vel, const float *kappa_a,
                  const float *kappa_s, const float *eta, const lbrt_coupling_out *out,
                  void *stream) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (!I) return fail(LBRT_E_INVAL, "I is NULL");
  if (!out) return fail(LBRT_E_INVAL, "out is NULL");
  if (out->S && (!kappa_a || !kappa_s || !eta))
    return fail(LBRT_E_INVAL, "the sources S need kappa_a, kappa_s and eta");
  if (!out->E && !out->F && !out->P && !out->J && !out->H && !out->S) return LBRT_OK;
  const lbrt_desc &d = c->desc;
  CoupArgs a{};
  a.E = out->E;
  a.F = out->F;
  a.P = out->P;
  a.J = out->J;
  a.H = out->H;
  a.S = out->S;
  a.vel = vel;
  a.kappa_a = kappa_a;
  a.kappa_s = kappa_s;
  a.eta = eta;
  a.ks_factor = 1.0 - d.lambda_aniso / 9.0;
  a.ncell = (int64_t)d.nx * d.ny * d.nz;
  a.e_off = e_offset(d.storage, d.ndir, a.ncell);
  a.ndir = d.ndir;
  hipError_t e = launch_coupling(d.storage, I, c->coup_dev, a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lbrt_coupling");
  return LBRT_OK;
}

int lbrt_convert(lbrt_ctx *c, const void *src, int32_t src_storage, void *dst,
                 int32_t dst_storage, void *stream) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (!src || !dst) return fail(LBRT_E_INVAL, "src and dst are required");
  if (src_storage < LBRT_FP32 || src_storage > LBRT_FP16_SHIFTED ||
      dst_storage < LBRT_FP32 || dst_storage > LBRT_FP16_SHIFTED)
    return fail(LBRT_E_INVAL, "bad storage type");
  if (is_shifted(src_storage) && is_shifted(dst_storage))
    return fail(LBRT_E_UNSUPPORTED, "shifted to shifted: convert through FP32");
  const lbrt_desc &d = c->desc;
  const int64_t ncell = (int64_t)d.nx * d.ny * d.nz;
  const size_t sb = (size_t)state_bytes(src_storage, d.ndir, ncell);
  const size_t db = (size_t)state_bytes(dst_storage, d.ndir, ncell);
  const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
  if (a < b + db && b < a + sb) return fail(LBRT_E_INVAL, "src and dst overlap");
  // The context's scales apply to the reduced (BF16/FP16, shifted) endpoint.
  const int sh = is_shifted(src_storage) ? src_storage : dst_storage;
  hipError_t e = launch_convert(src, src_storage, dst, dst_storage, c->scales_dev,
                                c->weights_dev, d.ndir, ncell, e_offset(sh, d.ndir, ncell),
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lbrt_convert");
  return LBRT_OK;
}

int64_t lbrt_state_bytes(int32_t storage, int32_t ndir, int64_t ncell) {
  if (storage < LBRT_FP32 || storage > LBRT_FP16_SHIFTED || ndir < 0 || ncell < 0) return -1;
  return state_bytes(storage, ndir, ncell);
}

int64_t lbrt_state_e_offset(int32_t storage, int32_t ndir, int64_t ncell) {
  if (storage < LBRT_FP32 || storage > LBRT_FP16_SHIFTED || ndir < 0 || ncell < 0) return -1;
  return e_offset(storage, ndir, ncell);
}

int lbrt_stream_copy(const void *src, void *dst, int64_t bytes, void *stream) {
  if (!src || !dst) return fail(LBRT_E_INVAL, "src and dst are required");
  if (bytes < 0 || bytes % 16 != 0) return fail(LBRT_E_INVAL, "bytes = %lld: need a multiple of 16",
                                                (long long)bytes);
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(LBRT_E_INVAL, "src and dst must be 16-byte aligned");
  const char *a = static_cast<const char *>(src), *b = static_cast<const char *>(dst);
  if (a < b + bytes && b < a + bytes) return fail(LBRT_E_INVAL, "src and dst overlap");
  if (bytes == 0) return LBRT_OK;
  hipError_t e = launch_stream_copy(src, dst, bytes / 16, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lbrt_stream_copy");
  return LBRT_OK;
}

}  // extern "C"

struct lbrt_batch {
  int ndom = 0;
  BatchLauncher launch = nullptr;
  BatchPlan plan{};
  std::vector<long long> step_main, step_gen;   // blocks of each step's two launches
  // device allocations
  BatchDomain *dom = nullptr;
  int4 *tiles = nullptr;
  GenTile *gtiles = nullptr;
  long long *main_prefix = nullptr, *gen_prefix = nullptr;
  char *tabs = nullptr;
  int32_t *step_active = nullptr;
  InflowArgs *noinflow = nullptr;
};

extern "C" {

int lbrt_set_tiling(lbrt_ctx *c, int32_t tx, int32_t ty, int32_t zlen, int32_t zlen_general) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (tx <= 0 || ty <= 0 || tx * ty != kTileCells || (tx & (tx - 1)) != 0)
    return fail(LBRT_E_INVAL, "tile %d x %d: need tx * ty = %d with tx a power of two", tx, ty,
                (int)kTileCells);
  if (zlen <= 0 || zlen_general <= 0) return fail(LBRT_E_INVAL, "z-range lengths must be > 0");
  const lbrt_desc &d = c->desc;
  c->tile = TileShape{tx, ty};
  c->zlen = std::min(zlen, d.nz);
  c->zlen_general = zlen_general;
  int rc = plan_all(c);
  if (rc != LBRT_OK) return rc;
  KParams p = make_params(c);
  return ensure_partials(c, total_partials(p));
}

int lbrt_get_tiling(const lbrt_ctx *c, int32_t *tx, int32_t *ty, int32_t *zlen,
                    int32_t *zlen_general) {
  if (!c) return fail(LBRT_E_INVAL, "ctx is NULL");
  if (tx) *tx = c->tile.tx;
  if (ty) *ty = c->tile.ty;
  if (zlen) *zlen = c->zlen;
  if (zlen_general) *zlen_general = c->zlen_general;
  return LBRT_OK;
}

void lbrt_batch_destroy(lbrt_batch *b) {
  if (!b) return;
  void *ptrs[] = {b->dom, b->tiles, b->gtiles, b->tabs, b->main_prefix, b->gen_prefix,
                  b->step_active, b->noinflow};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  delete b;
}

int lbrt_batch_create(const lbrt_domain *domains, int32_t ndomains, lbrt_batch **out) {
  if (!out) return fail(LBRT_E_INVAL, "out is NULL");
  if (!domains || ndomains < 1) return fail(LBRT_E_INVAL, "need at least one domain");
  const lbrt_ctx *c0 = domains[0].ctx;
  if (!c0) return fail(LBRT_E_INVAL, "domains[0].ctx is NULL");
  for (int k = 0; k < ndomains; ++k) {
    const lbrt_domain &D = domains[k];
    if (!D.ctx) return fail(LBRT_E_INVAL, "domains[%d].ctx is NULL", k);
    const lbrt_desc &d = D.ctx->desc;
    if (d.storage != c0->desc.storage || D.ctx->bucket != c0->bucket ||
        d.moving_fluid != c0->desc.moving_fluid)
      return fail(LBRT_E_INVAL, "domains[%d]: every domain needs the same storage, direction "
                  "bucket and fluid kind", k);
    if (!D.I_a || !D.I_b || D.I_a == D.I_b)
      return fail(LBRT_E_INVAL, "domains[%d]: two distinct population buffers needed", k);
    if (!D.kappa_a || !D.kappa_s || !D.eta)
      return fail(LBRT_E_INVAL, "domains[%d]: kappa_a, kappa_s, eta required", k);
    if ((d.moving_fluid != 0) != (D.vel != nullptr))
      return fail(LBRT_E_INVAL, "domains[%d]: vel must be given iff the fluid moves", k);
    if (D.nsteps < 0) return fail(LBRT_E_INVAL, "domains[%d].nsteps = %d < 0", k, D.nsteps);
  }
  BatchLauncher bl = batch_launcher(c0->desc.storage, c0->bucket, c0->desc.moving_fluid != 0);
  if (!bl)
    return fail(LBRT_E_UNSUPPORTED, "no batched kernel for storage %d with %d directions (%s)",
                c0->desc.storage, c0->desc.ndir, c0->desc.moving_fluid ? "moving" : "static");
  // order: longest run first, so that the domains active at any step are a prefix
  std::vector<int> order(ndomains);
  for (int k = 0; k < ndomains; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return domains[a].nsteps > domains[b].nsteps; });
  std::vector<BatchDomain> dom(ndomains);
  std::vector<int4> tiles;
  std::vector<GenTile> gtiles;
  std::vector<long long> mprefix(ndomains + 1, 0), gprefix(ndomains + 1, 0);
  std::vector<size_t> tile_start(ndomains), gtile_start(ndomains), tab_start(ndomains);
  size_t tab_total = 0;
  for (int j = 0; j < ndomains; ++j) {
    const lbrt_domain &D = domains[order[j]];
    const lbrt_ctx *c = D.ctx;
    // the batched kernels run the interior on the main kernel (plan mode 0)
    KParams p = make_params(c, 0);
    tile_start[j] = tiles.size();
    for (int zr = p.main_zr0; zr < p.main_zr0 + p.main_nzr; ++zr)
      for (int ty = p.main_ty0; ty < p.main_ty0 + p.main_nty; ++ty)
        for (int tx = 0; tx < p.ntx; ++tx) {
          const int zb = zr * p.zlen;
          tiles.push_back(make_int4(tx * p.tx, ty * p.ty, zb, std::min(p.nz, zb + p.zlen)));
        }
    const int32_t nmain = (int32_t)(tiles.size() - tile_start[j]);
    gtile_start[j] = gtiles.size();
    for (const GenTile &g : c->plan[0][0].general) gtiles.push_back(g);
    const int32_t ngen = (int32_t)(gtiles.size() - gtile_start[j]);
    BatchDomain &B = dom[j];
    B.p = p;
    B.p.flags &= ~(uint32_t)(KF_DIAG | KF_WRITE_EF | KF_XGHOSTS);
    tab_start[j] = tab_total;
    tab_total += (c->tab_bytes + 255) / 256 * 256;
    B.ntiles = nmain + ngen;
    B.nmain = nmain;
    B.nsteps = D.nsteps;
    mprefix[j + 1] = mprefix[j] + nmain;
    gprefix[j + 1] = gprefix[j] + ngen;
  }
  const int maxsteps = domains[order[0]].nsteps;
  std::vector<int32_t> active(std::max(maxsteps, 1), 0);
  lbrt_batch *b = new lbrt_batch();
  b->ndom = ndomains;
  b->launch = bl;
  b->step_main.assign(std::max(maxsteps, 0), 0);
  b->step_gen.assign(std::max(maxsteps, 0), 0);
  for (int st = 0; st < maxsteps; ++st) {
    int a = 0;
    while (a < ndomains && domains[order[a]].nsteps > st) ++a;
    active[st] = a;
    b->step_main[st] = mprefix[a];
    b->step_gen[st] = gprefix[a];
    if (mprefix[a] > 0x7fffffffLL || gprefix[a] > 0x7fffffffLL) {
      delete b;
      return fail(LBRT_E_INVAL, "step %d of the batch has %lld + %lld tiles (too many)", st,
                  mprefix[a], gprefix[a]);
    }
  }
  hipError_t e = hipSuccess;
  auto up = [&](void **dst, const void *src, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(dst, std::max<size_t>(bytes, 8));
    if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  up((void **)&b->tiles, tiles.data(), sizeof(int4) * tiles.size());
  up((void **)&b->gtiles, gtiles.data(), sizeof(GenTile) * gtiles.size());
  // the domains' direction tables, one block
  if (e == hipSuccess) e = hipMalloc((void **)&b->tabs, std::max<size_t>(tab_total, 256));
  for (int j = 0; j < ndomains && e == hipSuccess; ++j) {
    const lbrt_ctx *c = domains[order[j]].ctx;
    e = hipMemcpy(b->tabs + tab_start[j], c->tab_dev, c->tab_bytes, hipMemcpyDeviceToDevice);
  }
  // buffer offsets are taken from the domain array's own device address
  if (e == hipSuccess) e = hipMalloc((void **)&b->dom, sizeof(BatchDomain) * dom.size());
  if (e == hipSuccess) {
    const char *g = reinterpret_cast<const char *>(b->dom);
    auto off = [&](const void *ptr) -> int64_t {
      return ptr ? (int64_t)(reinterpret_cast<const char *>(ptr) - g) : kNoBuffer;
    };
    for (int j = 0; j < ndomains; ++j) {
      const lbrt_domain &D = domains[order[j]];
      BatchDomain &B = dom[j];
      B.tiles = b->tiles + tile_start[j];
      B.gtiles = b->gtiles + gtile_start[j];
      B.tab = (int64_t)tab_start[j];
      B.I[0] = off(D.I_a);
      B.I[1] = off(D.I_b);
      B.ka = off(D.kappa_a);
      B.ks = off(D.kappa_s);
      B.eta = off(D.eta);
      B.vel = off(D.vel);
      B.E = off(D.E);
      B.F = off(D.F);
    }
    e = hipMemcpy(b->dom, dom.data(), sizeof(BatchDomain) * dom.size(), hipMemcpyHostToDevice);
  }
  up((void **)&b->main_prefix, mprefix.data(), sizeof(long long) * mprefix.size());
  up((void **)&b->gen_prefix, gprefix.data(), sizeof(long long) * gprefix.size());
  up((void **)&b->step_active, active.data(), sizeof(int32_t) * active.size());
  InflowArgs none;
  std::memset(&none, 0, sizeof(none));
  up((void **)&b->noinflow, &none, sizeof(none));
  if (e != hipSuccess) {
    const int rc = fail(e == hipErrorOutOfMemory ? LBRT_E_NOMEM : LBRT_E_HIP,
                        "lbrt_batch_create: %s", hipGetErrorString(e));
    lbrt_batch_destroy(b);
    return rc;
  }
  BatchPlan &bp = b->plan;
  bp.dom = b->dom;
  bp.main_prefix = b->main_prefix;
  bp.gen_prefix = b->gen_prefix;
  bp.step_active = b->step_active;
  bp.maxsteps = maxsteps;
  bp.noinflow = b->noinflow;
  bp.tabs = b->tabs;
  bp.gbase = reinterpret_cast<char *>(b->dom);
  *out = b;
  return LBRT_OK;
}

int lbrt_step_batched(lbrt_batch *b, void *stream) {
  if (!b) return fail(LBRT_E_INVAL, "batch is NULL");
  if (b->plan.maxsteps == 0) return LBRT_OK;
  hipError_t e = b->launch(b->plan, b->step_main.data(), b->step_gen.data(),
                           static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "lbrt_step_batched");
  return LBRT_OK;
}

}  // extern "C"
