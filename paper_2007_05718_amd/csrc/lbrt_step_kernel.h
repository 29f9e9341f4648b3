// Fused stream-and-collide kernel for gfx950.
//
// A block of 256 threads owns a tile of 64 cells (TX x TY x TZ, x fastest).
// Its four wave64s split the directions: wave q streams the q-th quarter of
// the direction slots for all 64 cells, one cell per lane, and keeps those
// streamed values in registers.  A step therefore reads each stored population
// once from HBM (the other seven taps of the trilinear pull hit L1/L2) and
// writes it once:
//   stream   trilinear pull of eq. (interp) from the 2x2x2 upwind cells,
//   moments  per-wave partial E*, F* (eq. moments_discrete), combined across
//            the four waves through LDS in a fixed order,
//   collide  per-cell closed form of the chosen collision (Sec. 3.3, App. B),
//            evaluated by every wave,
//   store    each wave its quarter of the new populations; wave 0 also E, F
//            and the energy sums.
// Splitting directions over waves (rather than cells over lanes) keeps every
// direction constant wave-uniform (scalar registers) and cuts the registers a
// thread needs for its streamed values by four, which is what lets enough
// waves stay resident to cover HBM latency.
//
// Boundaries: the x faces are resolved per lane inside the main path (a lane
// on a face re-targets its x-shifted taps to a wrapped or in-cell address and
// swaps in the vacuum or inflow ghost value), so only tiles whose y or z halo
// leaves the box, and ragged tiles, take the per-tap checked path.
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
  __device__ static T ld(const float *p) { return *p; }
  __device__ static void st(float *p, T v) { __builtin_nontemporal_store(v, p); }
};

template <> struct StoreTraits<double> {
  using T = double;
  static constexpr bool kReduced = false;
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
  __device__ static T ld(const f16_t *p) {
    return (float)(*reinterpret_cast<const _Float16 *>(p));
  }
  __device__ static void st(f16_t *p, T v) {
    __builtin_nontemporal_store((_Float16)v, reinterpret_cast<_Float16 *>(p));
  }
};

template <typename S>
__device__ inline typename StoreTraits<S>::T ld_byte(const char *base, uint32_t byte_off) {
  return StoreTraits<S>::ld(reinterpret_cast<const S *>(base + byte_off));
}

template <typename T> __device__ inline T rcp(T x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// Block id -> tile.  Tiles are numbered along a sweep that keeps neighbours
// close in time: the box is cut into slabs of `slab` y-blocks; a slab is swept
// z-plane by z-plane, each plane y-block by y-block, x fastest.  The tile that
// needs a row of plane z-1 (or of the previous y-block) ran only a slab-plane
// earlier, so the row is still in L2.  The hardware deals block ids round-robin
// to the eight XCDs (each with its own L2); XCD x takes the x-th contiguous run
// of the sweep.
// ---------------------------------------------------------------------------
__device__ inline int xcd_tile(int bid, int ntiles) {
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return xcd * per + min(xcd, rem) + k;
}

__device__ inline void sweep_tile(int t, int ntx, int nty, int ntz, int slab, int &tix,
                                  int &tiy, int &tiz) {
  const int slab_tiles = ntx * slab * ntz;
  const int s = t / slab_tiles;
  int r = t - s * slab_tiles;
  const int yb0 = s * slab;
  const int nyb = min(slab, nty - yb0);   // the last slab may be thinner
  const int plane = ntx * nyb;
  tiz = r / plane;
  r -= tiz * plane;
  tiy = yb0 + r / ntx;
  tix = r - (r / ntx) * ntx;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum M per-thread values over the block; thread j < M writes out[j].
template <int M>
__device__ inline void block_sums(const double (&v)[M], double *out) {
  __shared__ double red[kBlock / 64][M];
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
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Checked stream of one direction at one in-box cell: periodic wrap, inflow
// ghosts (a point outside along exactly one axis) and vacuum elsewhere.
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ typename StoreTraits<S>::T
stream_checked(const S *__restrict__ P, const DirTab<typename StoreTraits<S>::T> &d, int x,
               int y, int z, int nx, int ny, int nz, int px, int py, int pz,
               const float *gx, const float *gy, const float *gz) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  T v[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    int cx = x - (b & 1) * d.s[0];
    int cy = y - ((b >> 1) & 1) * d.s[1];
    int cz = z - (b >> 2) * d.s[2];
    if (px) cx = cx < 0 ? cx + nx : (cx >= nx ? cx - nx : cx);
    if (py) cy = cy < 0 ? cy + ny : (cy >= ny ? cy - ny : cy);
    if (pz) cz = cz < 0 ? cz + nz : (cz >= nz ? cz - nz : cz);
    const bool ox = (unsigned)cx >= (unsigned)nx;
    const bool oy = (unsigned)cy >= (unsigned)ny;
    const bool oz = (unsigned)cz >= (unsigned)nz;
    const int nout = (int)ox + (int)oy + (int)oz;
    T val = T(0);
    if (nout == 0) {
      val = Tr::ld(P + ((int64_t)cz * ny + cy) * nx + cx);
    } else if (nout == 1) {
      const float *g = ox ? gx : (oy ? gy : gz);
      if (g != nullptr) {
        const int64_t gi = ox ? (int64_t)cz * ny + cy
                              : (oy ? (int64_t)cz * nx + cx : (int64_t)cy * nx + cx);
        const T gv = (T)g[gi];
        val = Tr::kReduced ? gv * d.inv_scale : gv;
      }
    }
    v[b] = val;
  }
  T acc = d.tw[0] * v[0];
#pragma unroll
  for (int b = 1; b < 8; ++b) acc = fma(d.tw[b], v[b], acc);
  if (Tr::kReduced) acc *= d.scale;
  return acc;
}

// ---------------------------------------------------------------------------
// Main-path helpers.  Lanes on an x face re-target the x-shifted taps to the
// wrapped cell (periodic) or to their own cell (vacuum or inflow; the value is
// replaced in main_interp), so every address stays in the box.
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ void main_load(const DirTab<typename StoreTraits<S>::T> &d,
                                          const char *base, uint32_t c0, bool at_lo, bool at_hi,
                                          bool perx, int nx, typename StoreTraits<S>::T (&v)[8]) {
  constexpr int SZ = (int)sizeof(S);
  const char *P = base + d.plane_off;
  const int s0 = d.s[0];
  const bool bad = s0 > 0 ? at_lo : (s0 < 0 ? at_hi : false);
  const int32_t adj = perx ? s0 * nx * SZ : s0 * SZ;
  const uint32_t c1 = c0 + (bad ? (uint32_t)adj : 0u);
#pragma unroll
  for (int b = 0; b < 8; ++b) v[b] = ld_byte<S>(P, ((b & 1) ? c1 : c0) + (uint32_t)d.off[b]);
}

template <typename S>
__device__ __forceinline__ typename StoreTraits<S>::T
main_interp(const DirTab<typename StoreTraits<S>::T> &d, bool at_lo, bool at_hi, bool perx,
            typename StoreTraits<S>::T (&v)[8]) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  // x-face lanes of non-periodic boxes: the x-shifted taps are ghosts; they
  // enter here as vacuum (0) and inflow ghost values are added afterwards by
  // x_ghost_correction
  const int s0 = d.s[0];
  const bool bad = !perx && (s0 > 0 ? at_lo : (s0 < 0 ? at_hi : false));
  v[1] = bad ? T(0) : v[1];
  v[3] = bad ? T(0) : v[3];
  v[5] = bad ? T(0) : v[5];
  v[7] = bad ? T(0) : v[7];
  T acc = d.tw[0] * v[0];
#pragma unroll
  for (int b = 1; b < 8; ++b) acc = fma(d.tw[b], v[b], acc);
  if (Tr::kReduced) acc *= d.scale;
  return acc;
}

// Inflow ghost values on an x face, for a lane on that face: the x-shifted
// taps read the face's ghost plane ([z][y] layout).  Every path computes I*
// with vacuum x ghosts first and adds this term, so all paths agree bit for bit.
// A tap that also leaves the box along y or z (an edge ghost) stays vacuum.
template <typename T>
__device__ __forceinline__ T x_ghost_correction(const DirTab<T> &d, const float *gx, int y,
                                                int z, int ny, int nz, int py, int pz) {
  T acc = T(0);
#pragma unroll
  for (int b = 1; b < 8; b += 2) {
    int cy = y - ((b >> 1) & 1) * d.s[1];
    int cz = z - (b >> 2) * d.s[2];
    if (py) cy = cy < 0 ? cy + ny : (cy >= ny ? cy - ny : cy);
    if (pz) cz = cz < 0 ? cz + nz : (cz >= nz ? cz - nz : cz);
    if ((unsigned)cy < (unsigned)ny && (unsigned)cz < (unsigned)nz)
      acc = fma(d.tw[b], (T)gx[(int64_t)cz * ny + cy], acc);
  }
  return acc;
}

// ---------------------------------------------------------------------------
// Per-slot moment accumulation, done as soon as a streamed value exists so
// that the interpolation of every slot completes in place (no long-lived taps).
//   static fluid: E* and F*, slots taken in pairs (a, b):
//       E += a + b,  F += n_a (a - b) + (n_a + n_b) b,
//     exact F-cancellation for antipodal pairs (n_a + n_b = 0), plain sums
//     otherwise;
//   moving fluid: E*, A = sum D_i^2 a_i I*_i and B = sum w_i a_i / D_i (App. B).
// ---------------------------------------------------------------------------
template <typename T>
struct Acc {
  T Es = T(0), F0 = T(0), F1 = T(0), F2 = T(0);  // static (F0..F2) or moving (F0 = A, F1 = B)
};

template <bool MOVING, int J, typename T>
__device__ __forceinline__ void accumulate(Acc<T> &m, const DirTab<T> *__restrict__ tb,
                                           const T *Is, T vx, T vy, T vz, T dtWk) {
  if constexpr (MOVING) {
    const DirTab<T> &d = tb[J];
    m.Es += Is[J];
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = rcp<T>(fma(dtWk, D, T(1)));
    m.F0 = fma(D * D * a, Is[J], m.F0);
    m.F1 = fma(d.w * a, rcp<T>(D), m.F1);
  } else if constexpr ((J & 1) == 1) {
    const DirTab<T> &da = tb[J - 1], &db = tb[J];
    const T a = Is[J - 1], b = Is[J];
    m.Es += a + b;
    const T dd = a - b;
    m.F0 = fma(da.n[0], dd, fma(da.n[0] + db.n[0], b, m.F0));
    m.F1 = fma(da.n[1], dd, fma(da.n[1] + db.n[1], b, m.F1));
    m.F2 = fma(da.n[2], dd, fma(da.n[2] + db.n[2], b, m.F2));
  }
}

// Unrolled loop helper: calls f.template operator()<J>() for J = 0..N-1.
template <int J, int N, typename F>
__device__ __forceinline__ void unroll(F &f) {
  if constexpr (J < N) {
    f.template operator()<J>();
    unroll<J + 1, N>(f);
  }
}

// ---------------------------------------------------------------------------
// The fused step.  NB direction slots (a multiple of 8, padded with null
// directions); wave q owns slots [q NB/4, (q+1) NB/4).
// ---------------------------------------------------------------------------
template <typename S, int NB, bool MOVING>
__global__ void __launch_bounds__(kBlock)
step_kernel(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
            const float *__restrict__ ks, const float *__restrict__ eta,
            const float *__restrict__ vel,
            const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams p,
            const InflowArgs *__restrict__ inflow, typename StoreTraits<S>::T *__restrict__ Eout,
            typename StoreTraits<S>::T *__restrict__ Fout, double *__restrict__ partials) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  constexpr int SZ = (int)sizeof(S);
  constexpr int M = NB / kWaves;
  static_assert(NB % (2 * kWaves) == 0, "direction slots must split into pairs per wave");

  const int nx = p.nx, ny = p.ny, nz = p.nz;
  int tix, tiy, tiz;
  sweep_tile(xcd_tile(blockIdx.x, p.ntiles), p.ntx, p.nty, p.ntz, p.slab, tix, tiy, tiz);
  const int x0 = tix * p.tx, y0 = tiy * p.ty, z0 = tiz * p.tz;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // direction quarter
  const int lane = threadIdx.x & 63;
  const int lx = lane % p.tx;
  const int ly = (lane / p.tx) % p.ty;
  const int lz = lane / (p.tx * p.ty);
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  const bool valid = x < nx && y < ny && z < nz;
  const uint32_t cell = valid ? (uint32_t)(x + nx * (y + ny * z)) : 0u;

  // Tiles whose y and z halos stay inside the box, with no ragged lanes, take
  // the main path; its x faces are handled per lane.
  const bool yz_inside = y0 >= 1 && z0 >= 1 && y0 + p.ty <= ny - 1 && z0 + p.tz <= nz - 1;
  const bool full_x = x0 + p.tx <= nx;
  const bool main_path = yz_inside && full_x;

  const T dt = (T)p.dt;
  T kat = T(0), kst = T(0), et = T(0);
  T vx = T(0), vy = T(0), vz = T(0);
  if (valid) {
    kat = (T)ka[cell];
    kst = (T)ks[cell];
    et = (T)eta[cell];
    if constexpr (MOVING) {
      vx = (T)vel[cell];
      vy = (T)vel[p.ncell + cell];
      vz = (T)vel[2 * p.ncell + cell];
    }
  }
  T W = T(1), dtWk = T(0);
  if constexpr (MOVING) {
    W = T(1) / sqrt(T(1) - (vx * vx + vy * vy + vz * vz));
    dtWk = dt * W * (kat + kst);
  }

  const DirTab<T> *__restrict__ tb = tab + q * M;   // this wave's slots
  T Is[M];
  Acc<T> m;

  if (main_path) {
    const char *base = reinterpret_cast<const char *>(Iin);
    const uint32_t c0 = cell * (uint32_t)SZ;
    const bool at_lo = x == 0, at_hi = x == nx - 1;
    const bool perx = p.periodic[0] != 0;
    T cur[8];
    main_load<S>(tb[0], base, c0, at_lo, at_hi, perx, nx, cur);
    // each slot prefetches the next slot's taps before interpolating its own
    auto body = [&]<int J>() {
      T nxt[8];
      if constexpr (J + 1 < M) main_load<S>(tb[J + 1], base, c0, at_lo, at_hi, perx, nx, nxt);
      Is[J] = main_interp<S>(tb[J], at_lo, at_hi, perx, cur);
      accumulate<MOVING, J>(m, tb, Is, vx, vy, vz, dtWk);
      if constexpr (J + 1 < M) {
#pragma unroll
        for (int b = 0; b < 8; ++b) cur[b] = nxt[b];
      }
    };
    unroll<0, M>(body);
  } else {
    const int px = p.periodic[0], py = p.periodic[1], pz = p.periodic[2];
    auto body = [&]<int J>() {
      const DirTab<T> &d = tb[J];
      T acc = T(0);
      if (valid) {
        const S *P = Iin + (int64_t)d.plane * p.ncell;
        const float *const *g = inflow->ghost[q * M + J];
        // x-face inflow ghosts come in through x_ghost_correction below
        acc = stream_checked<S>(P, d, x, y, z, nx, ny, nz, px, py, pz, nullptr, g[1], g[2]);
      }
      Is[J] = acc;
      accumulate<MOVING, J>(m, tb, Is, vx, vy, vz, dtWk);
    };
    unroll<0, M>(body);
  }
  if (p.flags & KF_XGHOSTS) {
    // Inflow ghosts on the x faces enter after the vacuum sums, slot by slot,
    // for the face lanes of the directions that have a ghost plane there.
    const bool xlo = valid && x == 0 && !p.periodic[0];
    const bool xhi = valid && x == nx - 1 && !p.periodic[0];
    auto body = [&]<int J>() {
      const DirTab<T> &d = tb[J];
      const float *gx = inflow->ghost[q * M + J][0];
      if (gx != nullptr && (d.s[0] > 0 ? xlo : (d.s[0] < 0 ? xhi : false))) {
        T dI = x_ghost_correction<T>(d, gx, y, z, ny, nz, p.periodic[1], p.periodic[2]);
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

  // Combine the four waves' partial sums in a fixed order,
  // (q0 + q1) + (q2 + q3), identical in every wave.
  __shared__ T red[kWaves][4][64];
  red[q][0][lane] = m.Es;
  red[q][1][lane] = m.F0;
  red[q][2][lane] = m.F1;
  red[q][3][lane] = m.F2;
  __syncthreads();
  auto comb = [&](int j) {
    return (red[0][j][lane] + red[1][j][lane]) + (red[2][j][lane] + red[3][j][lane]);
  };
  const T Es = comb(0), S0 = comb(1), S1 = comb(2), S2 = comb(3);

  T En = T(0), Fn0 = T(0), Fn1 = T(0), Fn2 = T(0);
  if constexpr (!MOVING) {
    const T F0 = S0, F1 = S1, F2 = S2;
    // Collision: every mode becomes I_i = c I*_i + w_i (alpha + n_i . beta).
    const T lam = (T)p.lam;
    T c, alpha, be0, be1, be2;
    if (p.mode == LBRT_COLL_EXPLICIT) {
      // eq. (collision-step) with I^eq and S of eq. (source-and-equil)
      c = T(1) - dt * (kst + kat);
      alpha = dt * (kst * Es + et);
      const T g = dt * kst * lam;
      be0 = g * F0; be1 = g * F1; be2 = g * F2;
      En = c * Es + alpha;
      Fn0 = c * F0 + be0 / T(3); Fn1 = c * F1 + be1 / T(3); Fn2 = c * F2 + be2 / T(3);
    } else if (p.mode == LBRT_COLL_LAMBDA) {
      // Lambda iteration: (E, F) <- moments of the decoupled solution, which
      // the rule's identities reduce to a scalar recursion per cell.
      c = T(1) / (T(1) + dt * (kst + kat));
      T Ek = Es, G0 = F0, G1 = F1, G2 = F2;
      const T h = dt * kst * lam / T(3);
      for (int it = 1; it < p.lambda_iters; ++it) {
        Ek = c * (Es + dt * (kst * Ek + et));
        G0 = c * (F0 + h * G0); G1 = c * (F1 + h * G1); G2 = c * (F2 + h * G2);
      }
      alpha = c * dt * (kst * Ek + et);
      const T g = c * dt * kst * lam;
      be0 = g * G0; be1 = g * G1; be2 = g * G2;
      En = c * Es + alpha;
      Fn0 = c * F0 + be0 / T(3); Fn1 = c * F1 + be1 / T(3); Fn2 = c * F2 + be2 / T(3);
    } else {
      // eq. (rte_implicit) solved exactly: the moment equations decouple to
      // E = (E* + dt eta)/(1 + dt ka), F = F*/(1 + dt(k0 + ka) - dt k0 lam/3).
      const T den = T(1) + dt * (kst + kat);
      c = T(1) / den;
      En = (Es + dt * et) / (T(1) + dt * kat);
      const T gF = T(1) / (den - dt * kst * lam / T(3));
      Fn0 = F0 * gF; Fn1 = F1 * gF; Fn2 = F2 * gF;
      alpha = c * dt * (kst * En + et);
      const T g = c * dt * kst * lam;
      be0 = g * Fn0; be1 = g * Fn1; be2 = g * Fn2;
    }
    if (valid) {
      if (p.flags & KF_LAMZERO) {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          if (q * M + j < p.ndir) {
            const DirTab<T> &d = tb[j];
            T o = fma(c, Is[j], d.w * alpha);
            if (Tr::kReduced) o *= d.inv_scale;
            Tr::st(Iout + (int64_t)d.plane * p.ncell + cell, o);
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < M; ++j) {
          if (q * M + j < p.ndir) {
            const DirTab<T> &d = tb[j];
            const T nb = alpha + d.n[0] * be0 + d.n[1] * be1 + d.n[2] * be2;
            T o = fma(c, Is[j], d.w * nb);
            if (Tr::kReduced) o *= d.inv_scale;
            Tr::st(Iout + (int64_t)d.plane * p.ncell + cell, o);
          }
        }
      }
    }
  } else {
    // Mixed-frame implicit collision (App. B): with D_i = 1 - v.n_i,
    // a_i = 1/(1 + dt W D_i (ka + k0)) and J = W^2 sum_i D_i^2 I_i (eq. J),
    //   J = (A + eta B) / (1 - k0 B),  A = W^2 sum D_i^2 a_i I*_i,
    //   B = (dt/W) sum w_i a_i / D_i,
    //   I_i = a_i [I*_i + dt w_i (eta + k0 J) / (W^3 D_i^3)].
    const T A = S0 * (W * W);
    const T B = S1 * (dt / W);
    const T J = (A + et * B) / (T(1) - kst * B);
    const T gam = dt * (et + kst * J) / (W * W * W);
    T e = T(0), f0 = T(0), f1 = T(0), f2 = T(0);
    if (valid) {
#pragma unroll
      for (int j = 0; j < M; ++j) {
        if (q * M + j < p.ndir) {
          const DirTab<T> &d = tb[j];
          const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
          const T a = rcp<T>(fma(dtWk, D, T(1)));
          const T iD = rcp<T>(D);
          const T o = a * fma(d.w * gam, iD * iD * iD, Is[j]);
          e += o;
          f0 = fma(d.n[0], o, f0);
          f1 = fma(d.n[1], o, f1);
          f2 = fma(d.n[2], o, f2);
          Tr::st(Iout + (int64_t)d.plane * p.ncell + cell, Tr::kReduced ? o * d.inv_scale : o);
        }
      }
    }
    // moments of the new state, combined like the streamed ones
    __syncthreads();
    red[q][0][lane] = e;
    red[q][1][lane] = f0;
    red[q][2][lane] = f1;
    red[q][3][lane] = f2;
    __syncthreads();
    En = comb(0); Fn0 = comb(1); Fn1 = comb(2); Fn2 = comb(3);
  }

  if (q == 0) {
    if (valid && (p.flags & KF_WRITE_EF)) {
      if (Eout) Eout[cell] = En;
      if (Fout) {
        Fout[cell] = Fn0;
        Fout[p.ncell + cell] = Fn1;
        Fout[2 * p.ncell + cell] = Fn2;
      }
    }
  }
  if (p.flags & KF_DIAG) {
    double v[kStepPartials];
    v[0] = (valid && q == 0) ? (double)En : 0.0;
    v[1] = (valid && q == 0) ? (double)Es : 0.0;
    block_sums<kStepPartials>(v, partials + (int64_t)blockIdx.x * kStepPartials);
  }
}

template <typename S, int NB, bool MOVING>
hipError_t launch_step(const void *Iin, void *Iout, const float *ka, const float *ks,
                       const float *eta, const float *vel, const void *tab, const KParams &p,
                       const InflowArgs *inflow, void *E, void *F, double *partials,
                       hipStream_t s) {
  using T = typename StoreTraits<S>::T;
  hipLaunchKernelGGL((step_kernel<S, NB, MOVING>), dim3(p.ntiles), dim3(kBlock), 0, s,
                     static_cast<const S *>(Iin), static_cast<S *>(Iout), ka, ks, eta, vel,
                     static_cast<const DirTab<T> *>(tab), p, inflow, static_cast<T *>(E),
                     static_cast<T *>(F), partials);
  return hipGetLastError();
}

}  // namespace lbrt
