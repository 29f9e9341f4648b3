// Fused stream-and-collide kernel for gfx950.
//
// One thread owns one cell and holds all N streamed populations of that cell
// in registers, so a step reads each stored population once from HBM (plus
// halo re-reads served by L2 / Infinity Cache) and writes it once:
//   stream   trilinear pull of eq. (interp) from the 2x2x2 upwind cells,
//   moments  E*, F* of the streamed populations (eq. moments_discrete),
//   collide  per-cell closed form of the chosen collision (Sec. 3.3, App. B),
//   store    the new populations, and optionally E, F and diagnostics.
// Blocks of 256 threads cover a TX x TY x TZ tile; block ids are remapped so
// that each of the eight XCDs (each with its own L2) sweeps one contiguous
// slab of tiles.  Tiles whose one-cell halo lies inside the box take a path
// without any boundary logic; the others resolve periodic wrap, vacuum and
// inflow ghosts per tap.
#pragma once

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

template <typename T> __device__ inline T rcp(T x);
template <> __device__ inline float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ inline double rcp<double>(double x) { return 1.0 / x; }

// ---------------------------------------------------------------------------
// Block-id -> tile: XCD x (x = bid mod 8) gets the x-th contiguous run of tiles.
// ---------------------------------------------------------------------------
__device__ inline int xcd_tile(int bid, int ntiles) {
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int xcd = bid & 7, k = bid >> 3;
  return xcd * per + min(xcd, rem) + k;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum kDiag per-thread values over the block; thread 0 writes them to out.
__device__ inline void block_diag(const double (&v)[kDiag], double *out) {
  __shared__ double red[kBlock / 64][kDiag];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kDiag; ++j) {
    const double s = wave_sum(v[j]);
    if (lane == 0) red[wv][j] = s;
  }
  __syncthreads();
  if (threadIdx.x < kDiag) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    out[threadIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// Checked stream of one direction at one in-box cell (boundary tiles).
// Returns I*_k in physical units; adds ghost inflow to *infl and this cell's
// outflux (of the incoming state) to outf[6] when diag is on.
// ---------------------------------------------------------------------------
template <typename S>
__device__ __attribute__((noinline)) typename StoreTraits<S>::T
stream_checked(const S *__restrict__ P, const DirTab<typename StoreTraits<S>::T> &d,
               int x, int y, int z, const KParams &p, const float *gx, const float *gy,
               const float *gz, bool diag, typename StoreTraits<S>::T *infl,
               typename StoreTraits<S>::T *outf) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;
  T v[8];
  T ghost_in = T(0);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    int cx = x - (b & 1) * d.s[0];
    int cy = y - ((b >> 1) & 1) * d.s[1];
    int cz = z - (b >> 2) * d.s[2];
    if (p.periodic[0]) cx = cx < 0 ? cx + p.nx : (cx >= p.nx ? cx - p.nx : cx);
    if (p.periodic[1]) cy = cy < 0 ? cy + p.ny : (cy >= p.ny ? cy - p.ny : cy);
    if (p.periodic[2]) cz = cz < 0 ? cz + p.nz : (cz >= p.nz ? cz - p.nz : cz);
    const bool ox = (unsigned)cx >= (unsigned)p.nx;
    const bool oy = (unsigned)cy >= (unsigned)p.ny;
    const bool oz = (unsigned)cz >= (unsigned)p.nz;
    const int nout = (int)ox + (int)oy + (int)oz;
    T val = T(0);
    if (nout == 0) {
      val = Tr::ld(P + ((int64_t)cz * p.ny + cy) * p.nx + cx);
    } else if (nout == 1) {
      const float *g = ox ? gx : (oy ? gy : gz);
      if (g != nullptr) {
        const int64_t gi = ox ? (int64_t)cz * p.ny + cy
                              : (oy ? (int64_t)cz * p.nx + cx : (int64_t)cy * p.nx + cx);
        const T gv = (T)g[gi];
        ghost_in += d.tw[b] * gv;
        val = Tr::kReduced ? gv * d.inv_scale : gv;
      }
    }
    v[b] = val;
  }
  T acc = d.tw[0] * v[0];
#pragma unroll
  for (int b = 1; b < 8; ++b) acc = fma(d.tw[b], v[b], acc);
  if (Tr::kReduced) acc *= d.scale;
  if (diag) {
    *infl += ghost_in;
    // Energy of this cell that the pull sends outside the box; a point outside
    // along several axes is booked on the first of x, y, z.
    const T v0 = Tr::kReduced ? v[0] * d.scale : v[0];
    T stay = T(1);
    const int n3[3] = {p.nx, p.ny, p.nz};
    const int c3[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int sa = d.s[a];
      if (sa != 0 && !p.periodic[a]) {
        const bool at = sa > 0 ? (c3[a] == n3[a] - 1) : (c3[a] == 0);
        if (at) {
          outf[2 * a + (sa > 0 ? 1 : 0)] += stay * d.delta[a] * v0;
          stay *= (T(1) - d.delta[a]);
        }
      }
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// The fused step.
// ---------------------------------------------------------------------------
template <typename S, int NB>
__global__ void __launch_bounds__(kBlock)
step_kernel(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
            const float *__restrict__ ks, const float *__restrict__ eta,
            const float *__restrict__ vel,
            const DirTab<typename StoreTraits<S>::T> *__restrict__ tab, const KParams p,
            const InflowArgs inflow, typename StoreTraits<S>::T *__restrict__ Eout,
            typename StoreTraits<S>::T *__restrict__ Fout, double *__restrict__ partials) {
  using Tr = StoreTraits<S>;
  using T = typename Tr::T;

  const int tile = xcd_tile(blockIdx.x, p.ntiles);
  const int tix = tile % p.ntx;
  const int rest = tile / p.ntx;
  const int tiy = rest % p.nty;
  const int tiz = rest / p.nty;
  const int x0 = tix * p.tx, y0 = tiy * p.ty, z0 = tiz * p.tz;
  const int t = threadIdx.x;
  const int lx = t % p.tx;
  const int ly = (t / p.tx) % p.ty;
  const int lz = t / (p.tx * p.ty);
  const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
  const bool valid = x < p.nx && y < p.ny && z < p.nz;
  const bool interior = x0 >= 1 && y0 >= 1 && z0 >= 1 && x0 + p.tx <= p.nx - 1 &&
                        y0 + p.ty <= p.ny - 1 && z0 + p.tz <= p.nz - 1;
  const uint32_t cell = valid ? (uint32_t)(x + p.nx * (y + p.ny * z)) : 0u;
  const bool diag = (p.flags & KF_DIAG) != 0;

  T Is[NB];
  T infl = T(0);
  T outf[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};

  if (interior) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const DirTab<T> &d = tab[k];
      const S *P = Iin + (int64_t)d.plane * p.ncell;
      T v[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const S *Pb = P + d.off[b];
        v[b] = Tr::ld(Pb + cell);
      }
      T acc = d.tw[0] * v[0];
#pragma unroll
      for (int b = 1; b < 8; ++b) acc = fma(d.tw[b], v[b], acc);
      if (Tr::kReduced) acc *= d.scale;
      Is[k] = acc;
    }
  } else {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const DirTab<T> &d = tab[k];
      T acc = T(0);
      if (valid && k < p.ndir) {
        const S *P = Iin + (int64_t)d.plane * p.ncell;
        const float *g[3] = {nullptr, nullptr, nullptr};
        for (int j = 0; j < inflow.n; ++j) {
          if (inflow.dir[j] != d.plane) continue;
          const int f = inflow.face[j];
          const int a = f >> 1;
          // axis a pulls from the low face when s > 0, from the high face when s < 0
          if ((d.s[a] > 0 && (f & 1) == 0) || (d.s[a] < 0 && (f & 1) == 1)) g[a] = inflow.ptr[j];
        }
        acc = stream_checked<S>(P, d, x, y, z, p, g[0], g[1], g[2], diag, &infl, outf);
      }
      Is[k] = acc;
    }
  }

  const T dt = (T)p.dt;
  T kat = T(0), kst = T(0), et = T(0);
  if (valid) {
    kat = (T)ka[cell];
    kst = (T)ks[cell];
    et = (T)eta[cell];
  }
  T En = T(0), Fn0 = T(0), Fn1 = T(0), Fn2 = T(0), Es = T(0);

  if (!(p.flags & KF_MOVING)) {
    // Moments of the streamed populations; antipodal pairs enter F as
    // differences so nearly isotropic cells do not cancel large terms.
    T F0 = T(0), F1 = T(0), F2 = T(0);
    if (p.flags & KF_PAIRED) {
#pragma unroll
      for (int k = 0; k < NB; k += 2) {
        const T a = Is[k], b = Is[k + 1];
        Es += a + b;
        const T dd = a - b;
        F0 = fma(tab[k].n[0], dd, F0);
        F1 = fma(tab[k].n[1], dd, F1);
        F2 = fma(tab[k].n[2], dd, F2);
      }
    } else {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        Es += Is[k];
        F0 = fma(tab[k].n[0], Is[k], F0);
        F1 = fma(tab[k].n[1], Is[k], F1);
        F2 = fma(tab[k].n[2], Is[k], F2);
      }
    }
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
        for (int k = 0; k < NB; ++k) {
          if (k < p.ndir) {
            const DirTab<T> &d = tab[k];
            T o = fma(c, Is[k], d.w * alpha);
            if (Tr::kReduced) o *= d.inv_scale;
            Tr::st(Iout + (int64_t)d.plane * p.ncell + cell, o);
          }
        }
      } else {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          if (k < p.ndir) {
            const DirTab<T> &d = tab[k];
            const T nb = alpha + d.n[0] * be0 + d.n[1] * be1 + d.n[2] * be2;
            T o = fma(c, Is[k], d.w * nb);
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
    T vx = T(0), vy = T(0), vz = T(0);
    if (valid) {
      vx = (T)vel[cell];
      vy = (T)vel[p.ncell + cell];
      vz = (T)vel[2 * p.ncell + cell];
    }
    const T W = T(1) / sqrt(T(1) - (vx * vx + vy * vy + vz * vz));
    const T dtWk = dt * W * (kat + kst);
    T A = T(0), B = T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const DirTab<T> &d = tab[k];
      Es += Is[k];
      const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
      const T a = rcp<T>(fma(dtWk, D, T(1)));
      A = fma(D * D * a, Is[k], A);
      B = fma(d.w * a, rcp<T>(D), B);
    }
    A *= W * W;
    B *= dt / W;
    const T J = (A + et * B) / (T(1) - kst * B);
    const T gam = dt * (et + kst * J) / (W * W * W);
    if (valid) {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < p.ndir) {
          const DirTab<T> &d = tab[k];
          const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
          const T a = rcp<T>(fma(dtWk, D, T(1)));
          const T iD = rcp<T>(D);
          const T o = a * fma(d.w * gam, iD * iD * iD, Is[k]);
          En += o;
          Fn0 = fma(d.n[0], o, Fn0);
          Fn1 = fma(d.n[1], o, Fn1);
          Fn2 = fma(d.n[2], o, Fn2);
          Tr::st(Iout + (int64_t)d.plane * p.ncell + cell, Tr::kReduced ? o * d.inv_scale : o);
        }
      }
    }
  }

  if (valid && (p.flags & KF_WRITE_EF)) {
    if (Eout) Eout[cell] = En;
    if (Fout) {
      Fout[cell] = Fn0;
      Fout[p.ncell + cell] = Fn1;
      Fout[2 * p.ncell + cell] = Fn2;
    }
  }
  if (diag) {
    double v[kDiag];
    v[0] = valid ? (double)En : 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) v[1 + f] = (double)outf[f];
    v[7] = (double)infl;
    v[8] = valid ? (double)Es : 0.0;
    block_diag(v, partials + (int64_t)blockIdx.x * kDiag);
  }
}

template <typename S, int NB>
hipError_t launch_step(const void *Iin, void *Iout, const float *ka, const float *ks,
                       const float *eta, const float *vel, const void *tab, const KParams &p,
                       const InflowArgs &inflow, void *E, void *F, double *partials,
                       hipStream_t s) {
  using T = typename StoreTraits<S>::T;
  hipLaunchKernelGGL((step_kernel<S, NB>), dim3(p.ntiles), dim3(kBlock), 0, s,
                     static_cast<const S *>(Iin), static_cast<S *>(Iout), ka, ks, eta, vel,
                     static_cast<const DirTab<T> *>(tab), p, inflow, static_cast<T *>(E),
                     static_cast<T *>(F), partials);
  return hipGetLastError();
}

}  // namespace lbrt
