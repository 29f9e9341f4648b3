// Fused stream-and-collide kernel for gfx950: a z-march over xy tiles.
//
// A block owns an xy tile of 64 cells (tx x ty, x fastest, one cell per lane)
// and marches it through a range of z-planes.  Its NW wave64s (8 for the
// 112-, 152- and 200-slot buckets, 4 below) split the direction slots: wave q
// streams the q-th share of the slots for the tile's 64 cells and keeps the
// streamed values in registers.
//
// The trilinear pull of eq. (interp) is separable.  With the plane value
//   P_i(x, y, z') = (1-dy)[(1-dx) I(x, y, z') + dx I(x-sx, y, z')]
//                 +   dy [(1-dx) I(x, y-sy, z') + dx I(x-sx, y-sy, z')],
// the streamed population is  I*_i(z) = (1-dz) P_i(z) + dz P_i(z - sz).
// Marching up in z, each (direction, plane) value P is computed once and
// carried in a register to the next plane: a direction with sz > 0 reuses
// P(z-1) from the previous plane and computes P(z); one with sz < 0 reuses P(z)
// and computes P(z+1).  A plane costs four row loads per direction (two rows,
// each unshifted and x-shifted), all at a wave-uniform base address plus the
// lane's byte offset, so the address arithmetic is scalar.
//
// Per plane:
//   stream   the wave's slots, P from 4 row loads (issued a few slots ahead),
//            I* from P and the carried plane;
//   moments  per-wave partial E*, F* (eq. moments_discrete), combined across
//            the waves through LDS in a fixed order;
//   collide  per-cell closed form of the chosen collision (Sec. 3.3, App. B),
//            evaluated by every wave;
//   store    each wave its share of the new populations; wave 0 also E, F.
// The next plane's medium and first taps go out between the collision and
// the stores.  Energy diagnostics (sums of E and E*, the outflux through each
// face and the influx from inflow ghosts) accumulate per lane over the march
// and end as per-block partials in FP64.
//
// Boundaries: x faces are resolved per lane (the x-shifted load of a face lane
// is re-targeted to the wrapped cell, or to its own cell and zeroed), planes
// outside the box in z come from the inflow ghost plane or are vacuum, and
// tiles whose y halo leaves the box take a per-tap checked path.  A ragged
// last tile in x reads its row's last cell on its extra lanes.  Inflow
// ghosts on x faces enter through a separate correction term after the
// vacuum sums, so every path computes the same value.
#pragma once

#include <utility>

#include "lbrt_internal.h"

namespace lbrt {

// ---------------------------------------------------------------------------
// Storage types
// ---------------------------------------------------------------------------
template <typename S> struct StoreTraits;

template <> struct StoreTraits<float> {
  using T = float;
  static constexpr bool kReduced = false;
  static constexpr bool kShifted = false;
  __device__ static T ld(const float *p) { return *p; }
  __device__ static void st(float *p, T v) { __builtin_nontemporal_store(v, p); }
};

template <> struct StoreTraits<double> {
  using T = double;
  static constexpr bool kReduced = false;
  static constexpr bool kShifted = false;
  __device__ static T ld(const double *p) { return *p; }
  __device__ static void st(double *p, T v) { __builtin_nontemporal_store(v, p); }
};

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <> struct StoreTraits<bf16_t> {
  using T = float;
  static constexpr bool kReduced = true;
  static constexpr bool kShifted = false;
  __device__ static T ld(const bf16_t *p) {
    return __uint_as_float((uint32_t)(*reinterpret_cast<const uint16_t *>(p)) << 16);
  }
  __device__ static void st(bf16_t *p, T v) {
    __builtin_nontemporal_store(f32_to_bf16_rne(v), reinterpret_cast<uint16_t *>(p));
  }
};

template <> struct StoreTraits<f16_t> {
  using T = float;
  static constexpr bool kReduced = true;
  static constexpr bool kShifted = false;
  __device__ static T ld(const f16_t *p) {
    return (float)(*reinterpret_cast<const _Float16 *>(p));
  }
  __device__ static void st(f16_t *p, T v) {
    __builtin_nontemporal_store((_Float16)v, reinterpret_cast<_Float16 *>(p));
  }
};

// Equilibrium-shifted 16-bit storage: the stored value is the deviation
// (I_i - w_i E) / s_i from the cell's isotropic equilibrium, E in FP32
// beside it.  In an optically thick cell I_i is close to w_i E, and the
// deviation (about 3 w_i n_i.F) keeps F to the format's relative precision
// where plain 16-bit storage rounds it away with I_i.  The pull is linear,
// so the streamed population is w_i E~_i + s_i d*_i, E~_i being E pulled
// along direction i (the same trilinear weights).
template <typename B, typename S> struct ShiftedTraits {
  using T = float;
  static constexpr bool kReduced = true;
  static constexpr bool kShifted = true;
  __device__ static T ld(const S *p) { return StoreTraits<B>::ld(reinterpret_cast<const B *>(p)); }
  __device__ static void st(S *p, T v) { StoreTraits<B>::st(reinterpret_cast<B *>(p), v); }
};
template <> struct StoreTraits<bf16s_t> : ShiftedTraits<bf16_t, bf16s_t> {};
template <> struct StoreTraits<f16s_t> : ShiftedTraits<f16_t, f16s_t> {};

// ---------------------------------------------------------------------------
// Stochastic rounding of 16-bit storage.  Round-to-nearest loses any
// per-step change smaller than half a unit in the last place: with 8 (BF16)
// or 11 (FP16) significant bits, a population that an absorbing cell dims by
// less than that per step keeps its value for ever.  Rounding up with the
// probability of the dropped fraction is exact in expectation.  gfx950
// converts with stochastic rounding in one instruction (v_cvt_sr_*_f32; it
// adds the high 16 (BF16) or 13 (FP16) of 32 random bits to the dropped
// part), driven by 32 random bits per element: a hash of the cell's index
// combined with the step's seed, then the exclusive or with a random constant
// of the direction's plane.  The seed goes through the hash: with a plain
// exclusive or, bits that two steps' seeds share would be equal for every
// element in both steps, which correlates an element's rounding with its own
// previous one and biases the run (measured: 6e-4 after 200 steps of slow
// decay).  Every kernel path draws the same bits for an element, so they
// keep giving the same values.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t cell_hash(uint32_t c) {
  c ^= c >> 16;
  c *= 0x7feb352du;
  c ^= c >> 15;
  c *= 0x846ca68bu;
  c ^= c >> 16;
  return c;
}

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

template <typename S> __device__ __forceinline__ uint16_t to16_sr(float v, uint32_t r);
template <> __device__ __forceinline__ uint16_t to16_sr<bf16_t>(float v, uint32_t r) {
  const s16x2 h = __builtin_amdgcn_cvt_sr_bf16_f32(s16x2{0, 0}, v, r, false);
  return (uint16_t)h.x;
}
template <> __device__ __forceinline__ uint16_t to16_sr<f16_t>(float v, uint32_t r) {
  const f16x2 h = __builtin_amdgcn_cvt_sr_f16_f32(f16x2{0, 0}, v, r, false);
  return __builtin_bit_cast(uint16_t, h.x);
}
template <> __device__ __forceinline__ uint16_t to16_sr<bf16s_t>(float v, uint32_t r) {
  return to16_sr<bf16_t>(v, r);
}
template <> __device__ __forceinline__ uint16_t to16_sr<f16s_t>(float v, uint32_t r) {
  return to16_sr<f16_t>(v, r);
}

// Store of a 16-bit population with stochastic rounding (random bits r).
template <typename S>
__device__ __forceinline__ void sto_sr(char *base, uint32_t byte_off, float v, uint32_t r) {
  __builtin_nontemporal_store(to16_sr<S>(v, r), reinterpret_cast<uint16_t *>(base + byte_off));
}

// Load at a wave-uniform base plus a lane's byte offset.
template <typename S>
__device__ __forceinline__ typename StoreTraits<S>::T ldo(const S *base, uint32_t byte_off) {
  return StoreTraits<S>::ld(
      reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + byte_off));
}

template <typename T> __device__ inline T rcp(T x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }

// a / b: FP32 by the hardware reciprocal and one Newton correction of the
// quotient (within one ulp of the rounded quotient), FP64 exactly rounded.
template <typename T> __device__ inline T div_fast(T a, T b);
template <> __device__ inline float div_fast<float>(float a, float b) {
  const float r = __builtin_amdgcn_rcpf(b);
  const float q = a * r;
  return fmaf(fmaf(-b, q, a), r, q);
}
template <> __device__ inline double div_fast<double>(double a, double b) { return a / b; }

// v, or +0 when `zero` is 1: a mask on the bits (wave-uniform operands stay
// scalar instructions; an arithmetic factor would be a vector conversion and
// multiply, a select with a table load on one side a branch).
template <typename T> __device__ __forceinline__ T zero_if(T v, int zero);
template <> __device__ __forceinline__ float zero_if<float>(float v, int zero) {
  return __uint_as_float(__float_as_uint(v) & ((uint32_t)zero - 1u));
}
template <> __device__ __forceinline__ double zero_if<double>(double v, int zero) {
  return __longlong_as_double(__double_as_longlong(v) & ((long long)zero - 1));
}

// The same (wave-uniform) integer, which the compiler must treat as a new
// value: loads at an offset made from it cannot be hoisted out of a loop or
// merged with loads at another copy of it.  (An integer, not a pointer: the
// pointer keeps its global address space and the loads stay scalar.)
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

// A lane's value, which the compiler must treat as new: an address made from
// it cannot be hoisted out of a loop (where it would hold a 64-bit VGPR pair
// for the whole loop).
__device__ __forceinline__ uint32_t opaque_lane(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Store at a wave-uniform base plus a lane's byte offset.
template <typename S>
__device__ __forceinline__ void sto(char *base, uint32_t byte_off, typename StoreTraits<S>::T v) {
  StoreTraits<S>::st(reinterpret_cast<S *>(base + byte_off), v);
}

// Unrolled loop helper: calls f.template operator()<J>() for J = 0..N-1.
template <int J, int N, typename F>
__device__ __forceinline__ void unroll(F &f) {
  if constexpr (J < N) {
    f.template operator()<J>();
    unroll<J + 1, N>(f);
  }
}

// Element i of an inflow ghost plane.  The plane pointers come from a table
// in device memory, where the compiler cannot see that they are global
// memory; the cast makes the load a global one (a flat load would also wait
// on the LDS/scalar counter).
__device__ __forceinline__ float gload(const float *p, int64_t i) {
  return ((const __attribute__((address_space(1))) float *)p)[i];
}

// w0 u + w1 v, in one fixed rounding order used by every path.
template <typename T>
__device__ __forceinline__ T lerp2(T w0, T w1, T u, T v) {
  return fma(w1, v, w0 * u);
}

// Plane value from its four taps (x, y), (x-sx, y), (x, y-sy), (x-sx, y-sy).
template <typename T>
__device__ __forceinline__ T interp4(const DirTab<T> &d, T a, T a1, T b, T b1) {
  return lerp2(d.wy[0], d.wy[1], lerp2(d.wx[0], d.wx[1], a, a1), lerp2(d.wx[0], d.wx[1], b, b1));
}

// ---------------------------------------------------------------------------
// Block id -> (x tile, y tile, z range).  The hardware deals block ids
// round-robin to the eight XCDs (each with its own L2).  Tiles are ordered x
// fastest, then y, then z range, in runs of `per_range` tiles (one z range);
// the blocks of a range are dispatched together, and within it XCD k takes
// the k-th contiguous eighth, so the blocks resident on one XCD hold
// neighbouring rows and share their y-halo rows in that XCD's L2, while the
// whole GPU works on one z range at a time.  (Giving each XCD a contiguous
// eighth of all tiles instead, i.e. z ranges of its own, measured 3 % slower
// on the 256^3 steps; dealing the tiles out with no XCD-aware order at all
// doubled the bytes the L2s fetch, yet cost the FP32 step under 1 %.)
// ---------------------------------------------------------------------------
__device__ inline int xcd_tile(int bid, int per_range) {
  const int zr = bid / per_range, i = bid - zr * per_range;
  const int per = per_range >> 3, rem = per_range & 7;
  const int xcd = i & 7, k = i >> 3;
  return zr * per_range + xcd * per + min(xcd, rem) + k;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum M per-thread values over a block of W waves; thread j < M writes out[j].
template <int M, int W = kWaves>
__device__ inline void block_sums(const double (&v)[M], double *out) {
  __shared__ double red[W][M];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const double s = wave_sum(v[j]);
    if (lane == 0) red[wv][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < M) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// Waves per block of the step kernels for a bucket of NB direction slots:
// about 14 slots per wave keeps a lane's streamed and carried values in
// registers without spilling.
// Waves per SIMD the main kernel is compiled for: the second argument of
// __launch_bounds__ is the minimum number of waves per execution unit (SIMD),
// which caps VGPRs at 512 / that.  Two 8-wave blocks per CU (4 waves per SIMD,
// 128 VGPRs) so that one block computes while the other waits for HBM; three
// 4-wave blocks (3 per SIMD) for the smaller buckets.  16-bit storage asks
// for 2: under the 128-VGPR cap the compiler packs two loaded 16-bit values
// per VGPR, which waits for every prefetched load as soon as it is issued;
// with the looser bound it still allocates under 128 VGPRs, unpacked.
// FP64 (the checking form) with 112 slots or more also asks for 2: its
// values take two VGPRs each and would spill under 128.
template <typename S>
constexpr int waves_per_simd(int nb) {
  return (sizeof(S) == 2 || (sizeof(S) == 8 && nb >= 112)) ? (nb >= 112 ? 2 : 3)
                                                             : (nb >= 112 ? 4 : 3);
}
// Main path: slots whose four taps are in flight ahead of the slot being
// interpolated, for M slots per wave (memory-level parallelism per wave;
// each costs 4 VGPRs: 4 ahead fit the 128-VGPR budget at M = 14, 3 at 19).
// FP64 taps take two VGPRs each, so FP64 keeps 2 slots ahead; the 16-bit
// forms (which need a few more VGPRs for their conversions) and the moving
// fluid keep 3, which holds them under 128 VGPRs without spills.
template <typename S, bool MOVING = false>
constexpr int pf_depth(int m) {
  const int d = sizeof(S) == 8 ? 2 : ((sizeof(S) == 2 || MOVING || m > 14) ? 3 : 4);
  return m < d ? m : d;
}

// Fixed-order pairwise sum of W per-wave values, ((v0 + v1) + (v2 + v3)) + ...
template <typename T, int W>
__device__ __forceinline__ T tree_sum(const T (&v)[W]) {
  if constexpr (W == 1) {
    return v[0];
  } else {
    T h[W / 2];
#pragma unroll
    for (int i = 0; i < W / 2; ++i) h[i] = v[2 * i] + v[2 * i + 1];
    return tree_sum<T, W / 2>(h);
  }
}

__device__ __forceinline__ int wrap(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

// ---------------------------------------------------------------------------
// Outflux booking of one population of a cell on a non-periodic face: the
// fraction dt |n^a| / dx of the population leaves through the face of axis a
// (eq. interp); leaving along several axes, the part outside in x is booked on
// the x face, of the rest the part outside in y on the y face, the rest on the
// z face.  zlo/zhi: the cell's plane is the low/high z face.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void book_outflux(const DirTab<T> &d, T own, bool lox, bool hix,
                                             bool loy, bool hiy, bool zlo, bool zhi, T &fx, T &fy,
                                             T &fzlo, T &fzhi) {
  T stay = T(1);
  const bool lx = d.s[0] > 0 ? hix : (d.s[0] < 0 ? lox : false);
  fx += lx ? d.delta[0] * own : T(0);
  stay = lx ? d.wx[0] : stay;
  const bool ly = d.s[1] > 0 ? hiy : (d.s[1] < 0 ? loy : false);
  fy += ly ? stay * d.delta[1] * own : T(0);
  stay = ly ? stay * d.wy[0] : stay;
  const T oz = stay * d.delta[2] * own;
  fzhi += (d.s[2] > 0 && zhi) ? oz : T(0);
  fzlo += (d.s[2] < 0 && zlo) ? oz : T(0);
}

// ---------------------------------------------------------------------------
// Plane value on the checked path: plane zl inside the box; each of the four
// taps is wrapped on periodic axes, read inside the box, taken from the y-face
// inflow ghost plane ([z][x] layout) when it is outside in y only, and vacuum
// otherwise (x-face ghosts enter later through x_ghost_correction).  `own`
// gets the unshifted tap (the cell's own stored value).
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ typename StoreTraits<S>::T
checked_P(const DirTab<typename StoreTraits<S>::T> &d, const S *__restrict__ pl, int x, int y,
          bool valid, int nx, int ny, int perx, int pery, const float *gy, int zl,
          typename StoreTraits<S>::T &own) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  // The in-box loads of the four taps go out together (a tap outside the
  // box, or of an invalid lane, reads element 0 of the plane and is
  // replaced afterwards), so that a slot costs one wait, not four.
  T v[4];
  int gx[4];
  bool inb[4], yg[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int cx = x - (b & 1) * d.s[0];
    int cy = y - (b >> 1) * d.s[1];
    if (perx) cx = wrap(cx, nx);
    if (pery) cy = wrap(cy, ny);
    const bool ox = (unsigned)cx >= (unsigned)nx;
    const bool oy = (unsigned)cy >= (unsigned)ny;
    inb[b] = valid && !ox && !oy;
    yg[b] = valid && oy && !ox && gy != nullptr;
    gx[b] = cx;
    v[b] = Tr::ld(pl + (inb[b] ? (int64_t)cy * nx + cx : 0));
  }
  // Out-of-box taps, by selects (no per-lane branches): a slot with a
  // y-face ghost plane reads its four ghost values at clamped columns.
  T g[4] = {T(0), T(0), T(0), T(0)};
  if (gy != nullptr) {
#pragma unroll
    for (int b = 0; b < 4; ++b)
      g[b] = (T)gload(gy, (int64_t)zl * nx + min(max(gx[b], 0), nx - 1));
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const T gv = Tr::kReduced ? g[b] * d.inv_scale : g[b];
    v[b] = inb[b] ? v[b] : (yg[b] ? gv : T(0));
  }
  own = v[0];
  return interp4(d, v[0], v[1], v[2], v[3]);
}

// Equilibrium-shifted storage: the cell energy E of plane zl (FP32, [y][x])
// pulled with the same four taps and weights as checked_P.  A tap outside the
// box (after the periodic wrap) is a ghost: a ghost population enters whole
// through the deviation part, so its E part is 0.  `own` gets the unshifted
// tap.
template <typename T>
__device__ __forceinline__ T checked_PE(const DirTab<T> &d, const float *__restrict__ pl, int x,
                                        int y, bool valid, int nx, int ny, int perx, int pery,
                                        T &own) {
  T v[4];
  bool inb[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int cx = x - (b & 1) * d.s[0];
    int cy = y - (b >> 1) * d.s[1];
    if (perx) cx = wrap(cx, nx);
    if (pery) cy = wrap(cy, ny);
    inb[b] = valid && (unsigned)cx < (unsigned)nx && (unsigned)cy < (unsigned)ny;
    v[b] = (T)pl[inb[b] ? (int64_t)cy * nx + cx : 0];
  }
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (!inb[b]) v[b] = T(0);
  own = v[0];
  return interp4(d, v[0], v[1], v[2], v[3]);
}

// Plane value of a plane outside the box in z (non-periodic): taps inside the
// box in x and y read the z-face inflow ghost plane ([y][x] layout); all other
// taps are vacuum.
template <typename S>
__device__ __forceinline__ typename StoreTraits<S>::T
ghost_P(const DirTab<typename StoreTraits<S>::T> &d, const float *gz, int x, int y, bool valid,
        int nx, int ny, int perx, int pery) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  if (gz == nullptr || !valid) return T(0);
  T v[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int cx = x - (b & 1) * d.s[0];
    int cy = y - (b >> 1) * d.s[1];
    if (perx) cx = wrap(cx, nx);
    if (pery) cy = wrap(cy, ny);
    T val = T(0);
    if ((unsigned)cx < (unsigned)nx && (unsigned)cy < (unsigned)ny) {
      const T gv = (T)gload(gz, (int64_t)cy * nx + cx);
      val = Tr::kReduced ? gv * d.inv_scale : gv;
    }
    v[b] = val;
  }
  return interp4(d, v[0], v[1], v[2], v[3]);
}

// Inflow ghost values on an x face, for a lane on that face: the x-shifted
// taps read the face's ghost plane ([z][y] layout).  Every path computes I*
// with vacuum x ghosts first and adds this term, so all paths agree bit for
// bit.  A tap that also leaves the box along y or z (an edge ghost) stays
// vacuum.
template <typename T>
__device__ __forceinline__ T x_ghost_correction(const DirTab<T> &d, const float *gx, int y, int z,
                                                int ny, int nz, int py, int pz) {
  // The four taps are loaded together (an out-of-range tap reads element 0
  // and is skipped), so that they share one wait.
  float g[4];
  bool ok[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int b = 2 * k + 1;
    int cy = y - ((b >> 1) & 1) * d.s[1];
    int cz = z - (b >> 2) * d.s[2];
    if (py) cy = wrap(cy, ny);
    if (pz) cz = wrap(cz, nz);
    ok[k] = (unsigned)cy < (unsigned)ny && (unsigned)cz < (unsigned)nz;
    g[k] = gload(gx, ok[k] ? (int64_t)cz * ny + cy : 0);
  }
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (ok[k]) acc = fma(d.tw[2 * k + 1], (T)g[k], acc);
  return acc;
}

// Energy entering cell (x, y, z) from the inflow ghost plane g of a y or z
// face (axis a = 1 or 2): the taps shifted along a, with the other two
// coordinates inside the box (face layouts: y faces [z][x], z faces [y][x]).
template <typename T>
__device__ inline T ghost_influx(const DirTab<T> &d, const float *g, int a, int x, int y, int z,
                                 int nx, int ny, int nz, const int *per) {
  const int n3[3] = {nx, ny, nz};
  const int c3[3] = {x, y, z};
  const int o2 = a == 1 ? 2 : 1;   // the other non-x axis
  T acc = T(0);
  for (int b = 0; b < 8; ++b) {
    if (((b >> a) & 1) == 0) continue;
    int u = c3[0] - (b & 1) * d.s[0];
    int w = c3[o2] - ((b >> o2) & 1) * d.s[o2];
    if (per[0]) u = wrap(u, n3[0]);
    if (per[o2]) w = wrap(w, n3[o2]);
    if ((unsigned)u < (unsigned)n3[0] && (unsigned)w < (unsigned)n3[o2])
      acc = fma(d.tw[b], (T)gload(g, (int64_t)w * n3[0] + u), acc);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Per-slot moment accumulation, done as soon as a streamed value exists.
//   static fluid: E* and F*, slots taken in pairs (a, b):
//       E += a + b,  F += n_a (a - b) + (n_a + n_b) b,
//     exact F-cancellation for antipodal pairs (n_a + n_b = 0), plain sums
//     otherwise;
//   moving fluid: E*, A = sum D_i^2 a_i I*_i and B = sum w_i a_i / D_i (App. B).
// ---------------------------------------------------------------------------
// Per-lane moment sums of a wave's slots.  In an optically thick cell I_i is
// close to w_i E, so F = sum n_i I_i is a small difference of terms of size
// E, and plain FP32 partial sums would lose about eps_32 E of it.  The flux
// is therefore summed as residuals against an isotropic reference ref (the
// wave's first slot, I_0 / w_0):
//   sum_i n_i I_i = sum_i n_i (I_i - w_i ref) + ref sum_i n_i w_i,
// the residuals are O(F) in a thick cell, and the last term (the wave's
// sum of n_i w_i is a table constant) is added in FP64 when the waves'
// partial sums are combined.
template <typename T>
struct Acc {
  T Es = T(0), F0 = T(0), F1 = T(0), F2 = T(0);  // static (F0..F2) or moving (F0 = A, F1 = B)
  T ref = T(0);
};

template <bool MOVING, int J, int M, typename T>
__device__ __forceinline__ void accumulate(Acc<T> &m, const DirTab<T> *__restrict__ tb,
                                           const T *Is, T vx, T vy, T vz, T dtWk) {
  const DirTab<T> &d = tb[J];
  m.Es += Is[J];
  if constexpr (MOVING) {
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = rcp<T>(fma(dtWk, D, T(1)));
    m.F0 = fma(D * D * a, Is[J], m.F0);
    m.F1 = fma(d.w * a, rcp<T>(D), m.F1);
  } else {
    if constexpr (J == 0) m.ref = Is[0] * d.invw;
    const T r = fma(-d.w, m.ref, Is[J]);
    m.F0 = fma(d.n[0], r, m.F0);
    m.F1 = fma(d.n[1], r, m.F1);
    m.F2 = fma(d.n[2], r, m.F2);
  }
}

// ---------------------------------------------------------------------------
// Collision of a static fluid, per cell.  Every mode becomes
//   I_i = c I*_i + w_i (alpha + n_i . beta),
// and the new moments E', F' follow.  The E part (c, alpha, E') needs only E*
// and the F part (beta_a, F'_a) only F*_a, so the pair kernels compute them
// in different waves; both kernels call these functions, with explicit fused
// multiply-adds, so that they give the same bits for a cell.
//   implicit  eq. (rte_implicit) solved exactly: E' = (E* + dt eta)/(1 + dt ka),
//             F' = F*/(1 + dt (k0 + ka) - dt k0 lam/3);
//   explicit  eq. (collision-step) with I^eq and S of eq. (source-and-equil);
//   Lambda    `iters` cycles of the Lambda iteration: (E, F) <- moments of the
//             decoupled solution, which the rule's identities reduce to a
//             scalar recursion per cell.
// ---------------------------------------------------------------------------
template <typename T>
struct CoefE {
  T c, alpha, En;
};

template <typename T>
__device__ __forceinline__ CoefE<T> coef_E(int mode, int iters, T dt, T Es, T ka, T ks, T et) {
  CoefE<T> r;
  if (mode == LBRT_COLL_EXPLICIT) {
    r.c = fma(-dt, ks + ka, T(1));
    r.alpha = dt * fma(ks, Es, et);
    r.En = fma(r.c, Es, r.alpha);
  } else if (mode == LBRT_COLL_LAMBDA) {
    r.c = div_fast(T(1), fma(dt, ks + ka, T(1)));
    T Ek = Es;
    for (int it = 1; it < iters; ++it) Ek = r.c * fma(dt, fma(ks, Ek, et), Es);
    r.alpha = r.c * dt * fma(ks, Ek, et);
    r.En = fma(r.c, Es, r.alpha);
  } else {
    r.c = div_fast(T(1), fma(dt, ks + ka, T(1)));
    r.En = div_fast(fma(dt, et, Es), fma(dt, ka, T(1)));
    r.alpha = r.c * dt * fma(ks, r.En, et);
  }
  return r;
}

// One flux component: F'_a and beta_a (beta is 0 when lam == 0).
template <typename T>
__device__ __forceinline__ void coef_F(int mode, int iters, T dt, T lam, T F, T ka, T ks, T &Fn,
                                       T &beta) {
  const T third = T(1) / T(3);
  if (mode == LBRT_COLL_EXPLICIT) {
    const T c = fma(-dt, ks + ka, T(1));
    beta = dt * ks * lam * F;
    Fn = fma(beta, third, c * F);
  } else if (mode == LBRT_COLL_LAMBDA) {
    const T c = div_fast(T(1), fma(dt, ks + ka, T(1)));
    const T h = dt * ks * lam * third;
    T G = F;
    for (int it = 1; it < iters; ++it) G = c * fma(h, G, F);
    beta = c * dt * ks * lam * G;
    Fn = fma(beta, third, c * F);
  } else {
    const T den = fma(dt, ks + ka, T(1));
    const T c = div_fast(T(1), den);
    const T gF = div_fast(T(1), fma(-(dt * ks * lam), third, den));
    Fn = F * gF;
    beta = c * dt * ks * lam * Fn;
  }
}

// New population of one direction of a cell from its streamed value.
template <typename T>
__device__ __forceinline__ T collide_one(const DirTab<T> &d, T c, T alpha, T b0, T b1, T b2, T Is,
                                         bool lamzero) {
  if (lamzero) return fma(c, Is, d.w * alpha);
  const T nb = fma(d.n[2], b2, fma(d.n[1], b1, fma(d.n[0], b0, alpha)));
  return fma(c, Is, d.w * nb);
}

// ---------------------------------------------------------------------------
// The fused step.  NB direction slots (a multiple of 8, padded with null
// directions); wave q owns slots [q NB/NW, (q+1) NB/NW).  The tile is 64
// cells, 2^txlog wide in x; cells outside [0, xe) x [0, ye) are inactive.
// ---------------------------------------------------------------------------
template <typename S, int NB, bool MOVING, bool MAIN, int NW = waves_for(NB)>
__device__ __forceinline__ void
march(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
      const float *__restrict__ ks, const float *__restrict__ eta, const float *__restrict__ vel,
      const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams &p,
      const InflowArgs *__restrict__ inflow, typename StoreTraits<S>::T *__restrict__ Eout,
      typename StoreTraits<S>::T *__restrict__ Fout, double *__restrict__ partials, int x0,
      int y0, int zb, int ze, int txlog, int xe, int ye) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  constexpr int SZ = (int)sizeof(S);
  constexpr int M = NB / NW;
  static_assert(NB % NW == 0, "direction slots must split evenly over the waves");
  // Equilibrium-shifted storage: the states' FP32 E arrays (byte offset
  // e_off in each state buffer); E element offsets are twice the 16-bit ones.
  constexpr bool SH = Tr::kShifted;
  static_assert(!(SH && MOVING), "shifted storage: static fluid only");
  const char *const ein_bytes = reinterpret_cast<const char *>(Iin) + (SH ? p.e_off : 0);
  char *const eout_bytes = reinterpret_cast<char *>(Iout) + (SH ? p.e_off : 0);
  static_assert(NB / NW <= 32, "a wave's slots must fit a 32-bit mask");

  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int64_t pc = (int64_t)nx * ny;   // cells per z-plane
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // this wave's share
  const int lane = threadIdx.x & 63;
  const int perx = p.periodic[0], pery = p.periodic[1], perz = p.periodic[2];

  const int tx = 1 << txlog, ty = kTileCells >> txlog;
  const int x = x0 + (lane & (tx - 1));
  const int y = y0 + (lane >> txlog);
  const bool valid = x < xe && y < ye;
  // Byte offsets in a plane: the lane's cell, and its x-shifted tap x - sx
  // for sx > 0 / sx < 0; on a face lane the wrapped cell (periodic) or the
  // lane's own cell (a vacuum/inflow ghost: zeroed).  All offsets stay inside
  // the plane.
  // A ragged lane (x >= nx; main tiles are full in y) reads its row's last
  // cell, so that every tap it loads stays inside the box; its values are
  // never stored or summed.  General tiles send invalid lanes to cell 0.
  const uint32_t o0 = valid ? (uint32_t)(x + nx * y) * (uint32_t)SZ
                            : (MAIN ? (uint32_t)((nx - 1) + nx * y) * (uint32_t)SZ : 0u);
  const bool at0 = valid && x == 0, at1 = valid && x == nx - 1;
  uint32_t oxp = at0 ? (perx ? o0 + (uint32_t)((nx - 1) * SZ) : o0) : o0 - (uint32_t)SZ;
  uint32_t oxm = at1 ? (perx ? o0 - (uint32_t)((nx - 1) * SZ) : o0) : o0 + (uint32_t)SZ;
  if (!valid) oxp = oxm = o0;
  const bool lox = at0 && !perx, hix = at1 && !perx;   // on a non-periodic x face
  const bool loy = valid && y == 0 && !pery, hiy = valid && y == ny - 1 && !pery;
  // Main path, per lane: 1 where the x-shifted tap of a direction with
  // sx > 0 / sx < 0 is a vacuum or inflow ghost (zeroed), and 1 where such a
  // direction leaves through the lane's face (outflux weight).  A slot's
  // factor is sum over the two signs of (slot's sign factor) * (lane value):
  // plain FMAs with uniform operands, no per-slot lane masks.
  const T xzp = lox ? T(1) : T(0), xzm = hix ? T(1) : T(0);
  const T xop = hix ? T(1) : T(0), xom = lox ? T(1) : T(0);

  const bool diag = (p.flags & KF_DIAG) != 0;
  const bool xface_tile = !perx && (x0 == 0 || x0 + tx >= nx);
  const bool face_tile = xface_tile || (!pery && (y0 == 0 || y0 + ty >= ny));

  // This wave's slots.  Every plane re-reads them (scalar cache hits)
  // through an opaque copy of the pointer: hoisted out of the z loop, they
  // would keep hundreds of uniform values live in SGPRs and spill them.  One
  // copy of the table keeps its footprint within the scalar cache.
  const DirTab<T> *__restrict__ tb = tab + q * M;
  const T dt = (T)p.dt;

  // Diagnostics, per lane: sums of E and E* (wave 0), outflux through the
  // lane's x and y faces, influx (z faces: a separate kernel).
  double sE = 0.0, sEs = 0.0, fin = 0.0;
  T fx = T(0), fy = T(0);

  // Plane value of slot d (processing slot index `slot`) at plane zl by the
  // general rules: a plane outside the box in z is the z ghost plane (or
  // vacuum), otherwise each tap is checked.  With `book` (zl is one of this
  // block's planes) the own value is booked as x/y-face outflux.
  // Shifted storage: PE gets E pulled along the slot (0 for a ghost plane).
  auto general_P = [&](const DirTab<T> &d, int slot, int zl, bool book, T &PE) -> T {
    PE = T(0);
    if ((unsigned)zl >= (unsigned)nz)
      return ghost_P<S>(d, inflow->ghost[slot][2], x, y, valid, nx, ny, perx, pery);
    T own;
    const S *pl = Iin + (d.plane_off / SZ) + (int64_t)zl * pc;
    const T P = checked_P<S>(d, pl, x, y, valid, nx, ny, perx, pery, inflow->ghost[slot][1], zl,
                             own);
    T ownE = T(0);
    if constexpr (SH)
      PE = checked_PE<T>(d, reinterpret_cast<const float *>(ein_bytes) + (int64_t)zl * pc, x, y,
                         valid, nx, ny, perx, pery, ownE);
    // (an invalid lane has no face flags set and books 0)
    if (diag && book && face_tile) {
      T fz = T(0);
      T ownp = Tr::kReduced ? own * d.scale : own;
      if constexpr (SH) ownp = fma(d.w, ownE, ownp);
      book_outflux(d, ownp, lox, hix, loy, hiy, false, false, fx, fy, fz, fz);
    }
    return P;
  };
  // Main-path loads of the four taps of slot d from the z-plane that starts
  // at byte `plane` of the first direction's storage: rows y and y - sy, each
  // unshifted and x-shifted.  The x-shifted offset is o0 plus the lane's
  // delta for the slot's sign of sx, selected with the slot's all-ones/zero
  // masks.  The row addresses are two 64-bit scalar adds per slot.
  const uint32_t dxp = oxp - o0, dxm = oxm - o0;
  const char *const in_bytes = reinterpret_cast<const char *>(Iin);
  auto load4 = [&](const DirTab<T> &d, const char *plane, T (&v)[4]) {
    const char *b0 = plane + d.plane_off;
    const S *r0 = reinterpret_cast<const S *>(b0);
    const S *r1 = reinterpret_cast<const S *>(b0 + d.row_off);
    const uint32_t a0 = o0;
    const uint32_t ax = a0 + (dxp & d.mxp) + (dxm & d.mxm);
    v[0] = ldo<S>(r0, a0);
    v[1] = ldo<S>(r0, ax);
    v[2] = ldo<S>(r1, a0);
    v[3] = ldo<S>(r1, ax);
  };
  // Shifted storage: the same four taps of the E array at plane byte `plane`
  // (FP32: every byte offset doubles).
  auto load4E = [&](const DirTab<T> &d, const char *plane, T (&v)[4]) {
    const float *r0 = reinterpret_cast<const float *>(plane);
    const float *r1 = reinterpret_cast<const float *>(plane + 2 * d.row_off);
    const uint32_t a0 = 2u * o0;
    const uint32_t ax = a0 + ((2u * dxp) & d.mxp) + ((2u * dxm) & d.mxm);
    v[0] = (T)ldo<float>(r0, a0);
    v[1] = (T)ldo<float>(r0, ax);
    v[2] = (T)ldo<float>(r1, a0);
    v[3] = (T)ldo<float>(r1, ax);
  };
  // factor of the x-shifted taps of slot d for this lane (0 at a ghost)
  auto xkeep = [&](const DirTab<T> &d) {
    return fma(-d.cxp, xzp, fma(-d.cxm, xzm, T(1)));
  };
  // The new plane of a slot at output plane z (wrapped on a periodic z axis;
  // outside [0, nz) it is a z ghost plane), and whether it is one of this
  // block's own planes (own values are booked as outflux exactly once).
  auto new_plane = [&](const DirTab<T> &d, int z) {
    int zl = z + (d.s[2] < 0 ? 1 : 0);
    if (perz) zl = wrap(zl, nz);
    return zl;
  };
  auto own_plane = [&](const DirTab<T> &d, int z) { return d.s[2] >= 0 || z + 1 < ze; };

  // The slots of this wave with an inflow ghost plane on an x face that this
  // tile touches (bit J for slot J; only tiles on a non-periodic x face), so
  // that the plane loop tests one bit per slot instead of reading the slot's
  // ghost pointer and shift sign from memory on every plane.
  uint32_t xgmask = 0u;
  if ((p.flags & KF_XGHOSTS) && xface_tile) {
    const bool tlo = x0 == 0, thi = x0 + tx >= nx;
    auto scan = [&]<int J>() {
      const DirTab<T> &d = tab[q * M + J];
      if (inflow->ghost[q * M + J][0] != nullptr && ((d.s[0] > 0 && tlo) || (d.s[0] < 0 && thi)))
        xgmask |= 1u << J;
    };
    unroll<0, M>(scan);
  }

  // Prologue: the carried plane of every slot (P at zb - 1 for sz > 0, at zb
  // for sz < 0; nothing for sz == 0).  On the main path a plane outside the
  // box is vacuum (its clamped loads are weighted by 0).  Shifted storage
  // carries the plane value of the population itself, s_i P + w_i P_E (P_E:
  // E pulled along the slot), one register per slot.
  T carry[M];
  {
    auto pro = [&]<int J>() {
      const DirTab<T> &d = tb[J];
      carry[J] = T(0);
      if (d.s[2] != 0) {
        int zl = d.s[2] > 0 ? zb - 1 : zb;
        if (perz) zl = wrap(zl, nz);
        if constexpr (MAIN) {
          T v[4];
          const bool in = (unsigned)zl < (unsigned)nz;
          const int zc = min(max(zl, 0), nz - 1);
          load4(d, in_bytes + (int64_t)zc * pc * SZ, v);
          const T k1 = xkeep(d);
          carry[J] = (in ? T(1) : T(0)) * interp4(d, v[0], v[1] * k1, v[2], v[3] * k1);
          const T ko = fma(d.cxp, xop, d.cxm * xom);
          if (diag && d.s[2] < 0) fx = fma(ko * d.dxs, v[0], fx);
          if constexpr (SH) {
            T e[4];
            load4E(d, ein_bytes + (int64_t)zc * pc * 4, e);
            const T PE = (in ? T(1) : T(0)) * interp4(d, e[0], e[1] * k1, e[2], e[3] * k1);
            carry[J] = fma(d.w, PE, carry[J] * d.scale);
            if (diag && d.s[2] < 0) fx = fma(ko * (d.delta[0] * d.w), e[0], fx);
          }
        } else {
          T PE;
          carry[J] = general_P(d, q * M + J, zl, d.s[2] < 0, PE);
          if constexpr (SH) carry[J] = fma(d.w, PE, carry[J] * d.scale);
        }
      }
    };
    unroll<0, M>(pro);
  }

  // the waves' partial sums per plane (double-buffered): E, three flux sums
  // and the wave's isotropic reference
  __shared__ T red[2][NW][5][64];
  // element offsets of the new planes of output plane z: z (sz >= 0) and the
  // plane above (sz < 0), clamped into the box on a non-periodic axis
  auto plane_above = [&](int z) {
    const int za = z + 1 < nz ? z + 1 : (perz ? 0 : nz - 1);
    return (int64_t)za * pc;
  };
  // Main path: the taps of slots [J, J + D) of the plane are in flight
  // while slot J is interpolated; the first D of the next plane go out
  // before the collision's stores.
  constexpr int D = pf_depth<S, MOVING>(M);
  T pf[M][4];
  auto issue_first = [&](int zn) {
    const char *const p0 = in_bytes + (int64_t)zn * pc * SZ;
    const char *const p1 = in_bytes + plane_above(zn) * SZ;
    auto one = [&]<int J>() { load4(tb[J], tb[J].dzn_a ? p1 : p0, pf[J]); };
    unroll<0, D>(one);
  };

  // Shifted storage, main path: every slot of a plane interpolates E at the
  // same few cells (the tile's rows y0 - 1 .. y0 + ty and columns x0 - 1 ..
  // x0 + tx of the plane and of the plane above), so the block stages those
  // rows of the E array in LDS once per plane, and a slot's four E taps are
  // LDS reads instead of four global loads.  Staged plane j of the range is
  // sp(j) = zb for j = 0, else the plane above zb + j - 1; plane z = zb + k
  // reads sp(k) and sp(k + 1) (ring buffers k % 3 and (k + 1) % 3).  sp(k + 3)
  // is loaded during plane k (with the next plane's first taps) and written
  // at the end of plane k + 1's slot loop, between the barriers that follow
  // the last reads of its buffer and precede its first.  Staged column c
  // holds cell x0 - 1 + c wrapped (periodic x) or clamped into the box: the
  // taps a face or ragged lane takes there are the ones the global path takes.
  constexpr bool STAGE = SH && MAIN;
  static_assert(!STAGE || NW * 64 >= kStagePos, "four waves stage the E rows");
  __shared__ float estage[STAGE ? 3 : 1][STAGE ? kStagePos : 1];
  const int srow = tx + 2;                               // staged cells per row
  const int eown = ((lane >> txlog) + 1) * srow + (lane & (tx - 1)) + 1;
  uint32_t soff = 0u;       // byte offset in an E plane of this lane's staged cell
  bool sok = false;         // the lane stages a cell (waves 0 .. 3)
  float spend = 0.0f;       // staged value in flight (loaded a plane ahead)
  int sb = 0;               // ring buffer of sp(k) for the current plane k
  auto stage_plane = [&](int j) -> int64_t {
    return j == 0 ? (int64_t)zb * pc : plane_above(zb + j - 1);
  };
  auto stage_load = [&](int j) {
    if (sok) spend = ldo<float>(reinterpret_cast<const float *>(ein_bytes) + stage_plane(j), soff);
  };
  auto stage_write = [&](int b) {
    if (sok) estage[b][q * 64 + lane] = spend;
  };
  if constexpr (STAGE) {
    const int pidx = q * 64 + lane;
    sok = pidx < (kTileCells / tx + 2) * srow;
    if (sok) {
      const int r = pidx / srow;
      int gx = x0 - 1 + (pidx - r * srow);
      gx = perx ? ((gx % nx) + nx) % nx : min(max(gx, 0), nx - 1);
      soff = (uint32_t)(gx + nx * (y0 - 1 + r)) * 4u;
    }
    if (zb < ze) {
      stage_load(0);
      stage_write(0);
      stage_load(1);
      stage_write(1);
      if (zb + 1 < ze) stage_load(2);
      __syncthreads();
    }
  }
  // the four E taps of slot d from ring buffer b0 (its new plane is z) or
  // b1 (the plane above): rows y and y - sy, unshifted and x-shifted
  auto lds4E = [&](const DirTab<T> &d, int b0, int b1, T (&v)[4]) {
    const float *e = &estage[d.dzn_a ? b1 : b0][0];
    const int xs = (int)(d.mxm & 1u) - (int)(d.mxp & 1u);
    const int ys = d.row_shift > 0 ? srow : (d.row_shift < 0 ? -srow : 0);
    v[0] = (T)e[eown];
    v[1] = (T)e[eown + xs];
    v[2] = (T)e[eown + ys];
    v[3] = (T)e[eown + ys + xs];
  };
  if constexpr (MAIN)
    if (zb < ze) issue_first(zb);

  // The medium of a plane (kappa_a, kappa_s, eta and, for a moving fluid,
  // the velocity) is loaded during the previous plane, so that its use
  // never waits for it.  Every lane's cell index is inside the box (invalid lanes
  // read a clamped cell whose values are never stored or summed), so the
  // loads need no guard: a guarded load into a zeroed register would make
  // the compiler drain all outstanding memory operations at the zeroing.
  // The loads take a uniform base (the plane's first cell, `cplane`) plus
  // the lane's byte offset, made opaque per plane like the stores' below.
  T med[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  const uint32_t ocell = o0 / (uint32_t)SZ;   // the lane's cell in a plane
  auto load_medium = [&](int64_t cplane, uint32_t om) {
    med[0] = (T)ldo<float>(ka + cplane, om);
    med[1] = (T)ldo<float>(ks + cplane, om);
    med[2] = (T)ldo<float>(eta + cplane, om);
    if constexpr (MOVING) {
      med[3] = (T)ldo<float>(vel + cplane, om);
      med[4] = (T)ldo<float>(vel + p.ncell + cplane, om);
      med[5] = (T)ldo<float>(vel + 2 * p.ncell + cplane, om);
    }
  };
  load_medium((int64_t)zb * pc, ocell * 4u);

  for (int z = zb; z < ze; ++z) {
    const int par = (z - zb) & 1;
    tb = tab + opaque(q * M);
    // this wave's slots that hold directions (null slots come last), opaque
    // per plane so that the per-slot tests are not hoisted as lane masks
    const int nv = opaque(p.ndir - q * M);
    const int64_t cz = (int64_t)z * pc;

    // this plane's medium, loaded during the previous plane; the next
    // plane's goes out once the collision has used this one (the last plane
    // reloads its own cells)
    const T kat = med[0], kst = med[1], et = med[2];
    const T vx = med[3], vy = med[4], vz = med[5];
    const int64_t cz_next = z + 1 < ze ? cz + pc : cz;
    const uint32_t om = opaque_lane(ocell * 4u);
    T W = T(1), dtWk = T(0);
    if constexpr (MOVING) {
      W = T(1) / sqrt(T(1) - (vx * vx + vy * vy + vz * vz));
      dtWk = dt * W * (kat + kst);
    }

    T Is[M];
    Acc<T> m;
    if constexpr (MAIN) {
      // the new planes: this one (sz >= 0) and the one above (sz < 0); a
      // plane above a non-periodic box is clamped into it and weighted 0
      const char *const p0 = in_bytes + cz * SZ;
      const char *const p1 = in_bytes + plane_above(z) * SZ;
      // shifted storage: ring buffers of this plane and of the plane above
      const int sb1 = sb == 2 ? 0 : sb + 1;
      T pfE[M][4];   // a slot's E taps, read from LDS one slot ahead
      // the plane above a non-periodic box is vacuum: weight 0
      const int gh = (!perz && z + 1 >= nz) ? 1 : 0;
      // the plane above the last plane of the range belongs to the next block
      const int lastz = z + 1 >= ze ? 1 : 0;
      // FACE: a tile on a non-periodic x face.  Its face lanes zero the
      // x-shifted taps that are ghosts, and the x-face outflux of the own
      // values is booked (used with diagnostics on).  Every other tile takes
      // the copy without either (for its lanes the factor is exactly 1, so
      // both copies give the same bits).  Slot J issues the loads of slot
      // J + D before interpolating its own.
      auto slot = [&]<int J, bool FACE>() {
        const DirTab<T> &d = tb[J];
        if constexpr (J + D < M) load4(tb[J + D], tb[J + D].dzn_a ? p1 : p0, pf[J + D]);
        if constexpr (SH) {
          if constexpr (J == 0) lds4E(d, sb, sb1, pfE[0]);
          if constexpr (J + 1 < M) lds4E(tb[J + 1], sb, sb1, pfE[J + 1]);
        }
        const T(&cur)[4] = pf[J];
        T c1 = cur[1], c3 = cur[3];
        T k1 = T(1), ko = T(0);
        if constexpr (FACE) {
          k1 = xkeep(d);
          c1 *= k1;
          c3 *= k1;
          // the plane above the range belongs to the next block
          ko = fma(d.cxp, xop, d.cxm * xom);
          const T dxs = zero_if(d.dxs, d.dzn & lastz);
          fx = fma(ko * dxs, cur[0], fx);
        }
        const T Pn = interp4(d, cur[0], c1, cur[2], c3);
        // the new plane above a non-periodic box is vacuum
        const T wn = zero_if(d.wz_new, d.dzn & gh);
        if constexpr (SH) {
          const T(&ce)[4] = pfE[J];
          const T PEn = interp4(d, ce[0], ce[1] * k1, ce[2], ce[3] * k1);
          if constexpr (FACE)
            fx = fma(ko * zero_if(d.delta[0] * d.w, d.dzn & lastz), ce[0], fx);
          const T Ph = fma(d.w, PEn, Pn * d.scale);
          Is[J] = fma(d.wz_old, carry[J], wn * Ph);
          carry[J] = Ph;
        } else {
          T sv = fma(d.wz_old, carry[J], wn * Pn);
          if (Tr::kReduced) sv *= d.scale;
          Is[J] = sv;
          carry[J] = Pn;
        }
        accumulate<MOVING, J, M>(m, tb, Is, vx, vy, vz, dtWk);
      };
      auto body_face = [&]<int J>() { slot.template operator()<J, true>(); };
      auto body = [&]<int J>() { slot.template operator()<J, false>(); };
      if (xface_tile)
        unroll<0, M>(body_face);
      else
        unroll<0, M>(body);
      if constexpr (STAGE) {
        // sp(k + 2), loaded during the previous plane, into the buffer that
        // plane k - 1 read last (k = z - zb)
        if (z + 1 < ze) stage_write(sb1 == 2 ? 0 : sb1 + 1);
      }
    } else {
      auto body = [&]<int J>() {
        const DirTab<T> &d = tb[J];
        T PEn;
        const T Pn = general_P(d, q * M + J, new_plane(d, z), own_plane(d, z), PEn);
        T sv;
        if constexpr (SH) {
          const T Ph = fma(d.w, PEn, Pn * d.scale);
          sv = fma(d.wz_old, carry[J], d.wz_new * Ph);
          carry[J] = Ph;
        } else {
          sv = fma(d.wz_old, carry[J], d.wz_new * Pn);
          if (Tr::kReduced) sv *= d.scale;
          carry[J] = Pn;
        }
        Is[J] = valid ? sv : T(0);
        accumulate<MOVING, J, M>(m, tb, Is, vx, vy, vz, dtWk);
      };
      unroll<0, M>(body);
    }
    if (xgmask != 0u) {
      // Inflow ghosts on the x faces enter after the vacuum sums, slot by
      // slot, for the face lanes of the directions with a ghost plane there.
      auto body = [&]<int J>() {
        const DirTab<T> &d = tb[J];
        const float *gx = inflow->ghost[q * M + J][0];
        if (((xgmask >> J) & 1u) && (d.s[0] > 0 ? lox : hix)) {
          const T dI = x_ghost_correction<T>(d, gx, y, z, ny, nz, pery, perz);
          fin += (double)dI;
          Is[J] += dI;
          m.Es += dI;
          if constexpr (MOVING) {
            const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
            const T a = rcp<T>(fma(dtWk, D, T(1)));
            m.F0 = fma(D * D * a, dI, m.F0);
          } else {
            m.F0 = fma(d.n[0], dI, m.F0);
            m.F1 = fma(d.n[1], dI, m.F1);
            m.F2 = fma(d.n[2], dI, m.F2);
          }
        }
      };
      unroll<0, M>(body);
    }
    if (!MAIN && diag && (loy || hiy)) {
      // influx from inflow ghost planes on the y faces (a runtime loop)
      for (int j = 0; j < M; ++j) {
        const DirTab<T> &d = tb[j];
        const float *g = inflow->ghost[q * M + j][1];
        const bool on = d.s[1] > 0 ? loy : (d.s[1] < 0 ? hiy : false);
        if (g != nullptr && on)
          fin += (double)ghost_influx<T>(d, g, 1, x, y, z, nx, ny, nz, p.periodic);
      }
    }

    // Combine the waves' partial sums in a fixed pairwise order, identical
    // in every wave.
    red[par][q][0][lane] = m.Es;
    red[par][q][1][lane] = m.F0;
    red[par][q][2][lane] = m.F1;
    red[par][q][3][lane] = m.F2;
    red[par][q][4][lane] = m.ref;
    __syncthreads();
    auto comb = [&](int b, int j) {
      T v[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) v[w] = red[b][w][j][lane];
      return tree_sum<T, NW>(v);
    };
    // flux a of a combine: the residual sums plus, in FP64 and in wave
    // order, sum over waves of ref_w (sum of n_i w_i over wave w's slots)
    const DirTab<T> *__restrict__ tz = tab + opaque(0);
    auto flux = [&](int b, int a) -> T {
      // (exactly the residual sum when every wave's sum of n_i w_i is 0;
      // the moving fluid keeps the one code path, measured faster for it)
      if constexpr (!MOVING)
        if (p.flags & KF_NWQZERO) return comb(b, 1 + a);
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s = fma((double)red[b][w][4][lane], tz[w * M].nwq[a], s);
      return (T)((double)comb(b, 1 + a) + s);
    };
    const T Es = comb(par, 0);
    const T EsT = Es;
    T S0, S1, S2;
    if constexpr (MOVING) {
      S0 = comb(par, 1);
      S1 = comb(par, 2);
      S2 = T(0);
    } else {
      S0 = flux(par, 0);
      S1 = flux(par, 1);
      S2 = flux(par, 2);
    }


    // The next plane's first loads go out before the collision's stores,
    // after the collision has read this plane's medium (loads complete in
    // issue order, so a read of the medium behind them would wait for them).
    auto issue_next = [&]() {
      if constexpr (MAIN)
        if (z + 1 < ze) issue_first(z + 1);
      if constexpr (STAGE)
        if (z + 2 < ze) stage_load(z - zb + 3);
    };

    // the new populations of plane z: a uniform base per slot plus the
    // lane's byte offset (made opaque so the per-lane 64-bit sum is not
    // hoisted out of the z loop)
    char *const outz = reinterpret_cast<char *>(Iout) + cz * SZ;
    const uint32_t ost = opaque_lane(o0);
    // The collision reads the table through another opaque pointer, so that
    // its loads are not merged with the streaming phase's (which would keep
    // those values live across the barrier).
    const DirTab<T> *__restrict__ tbc = tab + opaque(q * M);
    T En = T(0), Fn0 = T(0), Fn1 = T(0), Fn2 = T(0);
    if constexpr (!MOVING) {
      const T lam = (T)p.lam;
      const CoefE<T> ce = coef_E<T>(p.mode, p.lambda_iters, dt, EsT, kat, kst, et);
      T be0, be1, be2;
      coef_F<T>(p.mode, p.lambda_iters, dt, lam, S0, kat, kst, Fn0, be0);
      coef_F<T>(p.mode, p.lambda_iters, dt, lam, S1, kat, kst, Fn1, be1);
      coef_F<T>(p.mode, p.lambda_iters, dt, lam, S2, kat, kst, Fn2, be2);
      En = ce.En;
      const T c = ce.c, alpha = ce.alpha;
      load_medium(cz_next, om);
      issue_next();
      if (valid) {
        const bool lz = (p.flags & KF_LAMZERO) != 0;
        // shifted storage stores the deviation from w_i E' (E' this
        // plane's new E, stored beside it)
        auto shift = [&](const DirTab<T> &d, T o) -> T {
          if constexpr (SH) return (T)fma(-d.w, En, o);
          return o;
        };
        // one copy of the slot loop per (stochastic rounding, lambda = 0)
        // case and per whether the wave has null slots, so that no slot
        // branches on them
        auto store_all = [&]<bool SR, bool LZ, bool FULL>() {
          const uint32_t gr = SR ? cell_hash((uint32_t)(cz + ocell) ^ p.seed) : 0u;
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const DirTab<T> &d = tbc[j];
            if (FULL || j < nv) {   // a direction (null slots come last)
              T o = shift(d, collide_one(d, c, alpha, be0, be1, be2, Is[j], LZ));
              if constexpr (SR) {
                sto_sr<S>(outz + d.plane_off, ost, o * d.inv_scale, gr ^ d.rnd);
              } else {
                if (Tr::kReduced) o *= d.inv_scale;
                sto<S>(outz + d.plane_off, ost, o);
              }
            }
          }
        };
        auto store_w = [&]<bool SR, bool LZ>() {
          if (nv >= M)
            store_all.template operator()<SR, LZ, true>();
          else
            store_all.template operator()<SR, LZ, false>();
        };
        if (Tr::kReduced && (p.flags & KF_STOCH)) {
          if (lz)
            store_w.template operator()<true, true>();
          else
            store_w.template operator()<true, false>();
        } else if (lz) {
          store_w.template operator()<false, true>();
        } else {
          store_w.template operator()<false, false>();
        }
      }
    } else {
      // Mixed-frame implicit collision (App. B): with D_i = 1 - v.n_i,
      // a_i = 1/(1 + dt W D_i (ka + k0)) and J = W^2 sum_i D_i^2 I_i (eq. J),
      //   J = (A + eta B) / (1 - k0 B),  A = W^2 sum D_i^2 a_i I*_i,
      //   B = (dt/W) sum w_i a_i / D_i,
      //   I_i = a_i [I*_i + dt w_i (eta + k0 J) / (W^3 D_i^3)].
      // J in FP64: with kappa_a << kappa_s the denominator 1 - k0 B is a
      // small difference
      const double A = (double)S0 * (double)(W * W);
      const double B = (double)S1 * (double)(dt / W);
      const T J = (T)((A + (double)et * B) / (1.0 - (double)kst * B));
      const T gam = div_fast(dt * (et + kst * J), W * W * W);
      issue_next();
      T e = T(0), f0 = T(0), f1 = T(0), f2 = T(0), ref = T(0);
      const bool sr = Tr::kReduced && (p.flags & KF_STOCH);
      const uint32_t gr = sr ? cell_hash((uint32_t)(cz + ocell) ^ p.seed) : 0u;
      if (valid) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          const DirTab<T> &d = tbc[j];
          if (j < nv) {
            const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
            const T a = rcp<T>(fma(dtWk, D, T(1)));
            const T iD = rcp<T>(D);
            const T o = a * fma(d.w * gam, iD * iD * iD, Is[j]);
            // (flux as residuals against the wave's first slot, as above)
            if (j == 0) ref = o * d.invw;
            const T r = fma(-d.w, ref, o);
            e += o;
            f0 = fma(d.n[0], r, f0);
            f1 = fma(d.n[1], r, f1);
            f2 = fma(d.n[2], r, f2);
            if constexpr (Tr::kReduced) {
              if (sr) sto_sr<S>(outz + d.plane_off, ost, o * d.inv_scale, gr ^ d.rnd);
              else sto<S>(outz + d.plane_off, ost, o * d.inv_scale);
            } else {
              sto<S>(outz + d.plane_off, ost, o);
            }
          }
        }
      }
      load_medium(cz_next, om);
      // Moments of the new state, combined like the streamed ones through the
      // other half of the double buffer.  It is free: its last readers were
      // the previous plane's, and every wave has passed this plane's barrier.
      red[par ^ 1][q][0][lane] = e;
      red[par ^ 1][q][1][lane] = f0;
      red[par ^ 1][q][2][lane] = f1;
      red[par ^ 1][q][3][lane] = f2;
      red[par ^ 1][q][4][lane] = ref;
      __syncthreads();
      En = comb(par ^ 1, 0);
      Fn0 = flux(par ^ 1, 0);
      Fn1 = flux(par ^ 1, 1);
      Fn2 = flux(par ^ 1, 2);
      // The next plane writes red[par ^ 1] only after every wave has read it.
      __syncthreads();
    }

    if constexpr (SH) {
      // the new state's E, part of the shifted state (wave 0)
      if (q == 0 && valid)
        *reinterpret_cast<float *>(eout_bytes + cz * 4 + opaque_lane(ocell * 4u)) = (float)En;
    }
    if (q == 0 && valid) {
      if (p.flags & KF_WRITE_EF) {
        // at a uniform base plus the lane's (opaque) byte offset, as above
        const uint32_t oT = opaque_lane(ocell * (uint32_t)sizeof(T));
        auto put = [&](T *base, T v) {
          *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + oT) = v;
        };
        if (Eout) put(Eout + cz, En);
        if (Fout) {
          put(Fout + cz, Fn0);
          put(Fout + p.ncell + cz, Fn1);
          put(Fout + 2 * p.ncell + cz, Fn2);
        }
      }
      if (diag) {
        sE += (double)En;
        sEs += (double)Es;
      }
    }
    if constexpr (STAGE) sb = sb == 2 ? 0 : sb + 1;
  }

  if (diag) {
    // per-block partials: sum E, sum E*, outflux per face (-x,+x,-y,+y,-z,+z),
    // influx
    double v[kStepPartials];
    v[0] = sE;
    v[1] = sEs;
    v[2] = lox ? (double)fx : 0.0;
    v[3] = hix ? (double)fx : 0.0;
    v[4] = loy ? (double)fy : 0.0;
    v[5] = hiy ? (double)fy : 0.0;
    v[6] = 0.0;
    v[7] = 0.0;
    v[8] = fin;
    block_sums<kStepPartials, NW>(v, partials + (int64_t)blockIdx.x * kStepPartials);
  }
}

// The main kernel: tiles whose y halo stays inside the box, with no ragged
// lanes, in z ranges whose z ghost planes (if any) are vacuum.  Block id ->
// tile in the XCD-aware order of xcd_tile.
template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(64 * waves_for(NB), waves_per_simd<S>(NB))
step_kernel_main(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
                 const float *__restrict__ ks, const float *__restrict__ eta,
                 const float *__restrict__ vel,
                 const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams p,
                 const InflowArgs *__restrict__ inflow,
                 typename StoreTraits<S>::T *__restrict__ Eout,
                 typename StoreTraits<S>::T *__restrict__ Fout, double *__restrict__ partials) {
  const int t = xcd_tile(blockIdx.x, p.ntx * p.main_nty);
  const int tix = t % p.ntx;
  const int r = t / p.ntx;
  const int tiy = p.main_ty0 + r % p.main_nty;
  const int tzr = p.main_zr0 + r / p.main_nty;
  const int zb = tzr * p.zlen;
  march<S, NB, MOVING, true>(Iin, Iout, ka, ks, eta, vel, tab, p, inflow, Eout, Fout, partials,
                             tix * p.tx, tiy * p.ty, zb, min(p.nz, zb + p.zlen), p.txlog, p.nx,
                             p.ny);
}

// The general kernel: every other tile (y-face rows, ragged tiles, z ranges
// next to an inflow z face), in short z ranges, from a host-built list of
// (x0, y0, zb, ze).  Its partials follow the main kernel's.
template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(64 * waves_for(NB))
step_kernel_general(const S *__restrict__ Iin, S *__restrict__ Iout,
                    const float *__restrict__ ka, const float *__restrict__ ks,
                    const float *__restrict__ eta, const float *__restrict__ vel,
                    const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams p,
                    const InflowArgs *__restrict__ inflow,
                    typename StoreTraits<S>::T *__restrict__ Eout,
                    typename StoreTraits<S>::T *__restrict__ Fout, double *__restrict__ partials) {
  const GenTile &g = p.general_list[blockIdx.x];
  march<S, NB, MOVING, false>(Iin, Iout, ka, ks, eta, vel, tab, p, inflow, Eout, Fout,
                              partials + (int64_t)p.nblocks * kStepPartials, g.x0, g.y0, g.zb,
                              g.ze, g.txlog, g.xe, g.ye);
}

// ---------------------------------------------------------------------------
// Boundary energy fluxes through the z faces of the state entering a step
// (non-periodic z only), as per-block partials in the step kernel's format
// (columns 6 and 7: outflux through -z and +z; column 8: influx from z-face
// inflow ghost planes).  One thread per cell of the two face planes; the
// outflux of a cell that also lies on an x or y face is booked by the same
// rule as in the step kernel (the x and y parts there, the rest here).
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(kBlock)
zface_kernel(const S *__restrict__ I, const DirTab<typename StoreTraits<S>::T> *__restrict__ tab,
             const KParams p, const InflowArgs *__restrict__ inflow,
             double *__restrict__ partials) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int64_t pc = (int64_t)nx * ny;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;   // over 2 pc
  const int g = blockIdx.y;   // direction group: directions g, g + G, ...
  double v[kStepPartials];
#pragma unroll
  for (int j = 0; j < kStepPartials; ++j) v[j] = 0.0;
  if (k < 2 * pc) {
    const int face = k >= pc;   // 0: z = 0, 1: z = nz - 1
    const int64_t c = face ? k - pc : k;
    const int y = (int)(c / nx), x = (int)(c - (int64_t)y * nx);
    const int z = face ? nz - 1 : 0;
    const bool lox = !p.periodic[0] && x == 0, hix = !p.periodic[0] && x == nx - 1;
    const bool loy = !p.periodic[1] && y == 0, hiy = !p.periodic[1] && y == ny - 1;
    T out = T(0), in = T(0);
    for (int i = g; i < p.ndir; i += (int)gridDim.y) {
      const DirTab<T> &d = tab[i];
      const int sz = d.s[2];
      if (sz != 0 && (sz > 0) == (face == 1)) {
        // leaves through this face
        T own = Tr::ld(I + (d.plane_off / (int64_t)sizeof(S)) + (int64_t)z * pc + c);
        if (Tr::kReduced) own *= d.scale;
        if constexpr (Tr::kShifted)
          own = fma(d.w, (T)reinterpret_cast<const float *>(
                             reinterpret_cast<const char *>(I) + p.e_off)[(int64_t)z * pc + c],
                    own);
        T fx = T(0), fy = T(0), flo = T(0), fhi = T(0);
        book_outflux(d, own, lox, hix, loy, hiy, face == 0, face == 1, fx, fy, flo, fhi);
        out += flo + fhi;
      }
      const float *g = inflow->ghost[i][2];
      if (g != nullptr && sz != 0 && (sz > 0) == (face == 0))
        in += ghost_influx<T>(d, g, 2, x, y, z, nx, ny, nz, p.periodic);
    }
    v[6 + face] = (double)out;
    v[8] = (double)in;
  }
  block_sums<kStepPartials>(
      v, partials + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * kStepPartials);
}

}  // namespace lbrt

#include "lbrt_pair_kernel.h"

namespace lbrt {

template <typename S, int NB, bool MOVING>
hipError_t launch_step(const void *Iin, void *Iout, const float *ka, const float *ks,
                       const float *eta, const float *vel, const void *tab, const KParams &p,
                       const InflowArgs *inflow, void *E, void *F, double *partials,
                       hipStream_t s) {
  using T = typename StoreTraits<S>::T;
  // the general kernel first: its short blocks do not leave a tail
  if (p.ngeneral > 0)
    hipLaunchKernelGGL((step_kernel_general<S, NB, MOVING>), dim3(p.ngeneral),
                       dim3(64 * waves_for(NB)), 0,
                       s, static_cast<const S *>(Iin), static_cast<S *>(Iout), ka, ks, eta, vel,
                       static_cast<const DirTab<T> *>(tab), p, inflow, static_cast<T *>(E),
                       static_cast<T *>(F), partials);
  if constexpr (pair_kernel_exists<S, NB, MOVING>()) {
    if (p.pair) {
      if (p.nblocks > 0)
        hipLaunchKernelGGL((step_kernel_pair<S, NB>), dim3(p.nblocks), dim3(64 * waves_for(NB)),
                           0, s, static_cast<const S *>(Iin), static_cast<S *>(Iout), ka, ks, eta,
                           p.pair_tab, p.pair_coll, static_cast<const DirTab<float> *>(tab),
                           inflow, p, static_cast<float *>(E), static_cast<float *>(F),
                           partials);
      return hipGetLastError();
    }
  }
  if (p.nblocks > 0)
    hipLaunchKernelGGL((step_kernel_main<S, NB, MOVING>), dim3(p.nblocks),
                       dim3(64 * waves_for(NB)), 0, s,
                       static_cast<const S *>(Iin), static_cast<S *>(Iout), ka, ks, eta, vel,
                       static_cast<const DirTab<T> *>(tab), p, inflow, static_cast<T *>(E),
                       static_cast<T *>(F), partials);
  return hipGetLastError();
}

}  // namespace lbrt
