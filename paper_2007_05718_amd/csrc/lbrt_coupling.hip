// Per-cell moments of a stored state and the radiative sources that the
// coupling loop of Sec. 5 hands to a fluid code (its items 3 and 4):
//   E, F^j, P^jk           eqs. moments_discrete and higher_moments,
//   J, H_j                 eq. J (fluid-frame energy and flux densities),
//   H_0 = v^j H_j          the time component of H orthogonal to the fluid
//                          four-velocity (taken contravariantly, so that S_0
//                          is the energy the collision takes from the
//                          radiation),
//   S_0, S_j               W (ka J - eta) + k H_0 and W (ka J - eta) v_j + k H_j,
//                          k = ka + k_0 (1 - lambda / 9), i.e. k_s = k_0 - k_1 / 3.
//
// One thread per cell, directions in storage order, the ten sums in FP64:
// J and H are differences of terms of size W^2 E, which FP32 sums of 100+
// populations would not resolve in a fast, optically thin flow.  The pass
// is a stream over the state (ndir loads per cell, coalesced across the
// wave) with a few hundred FP64 operations per cell, so it is bound by HBM;
// eight directions' loads are issued before their sums to keep enough
// bytes in flight per wave.
#include "lbrt_step_kernel.h"

namespace lbrt {

namespace {

constexpr int kCoupBlock = 256;
constexpr int kCoupUnroll = 8;

template <typename O> __device__ __forceinline__ void put(void *base, int64_t k, double v) {
  __builtin_nontemporal_store((O)v, static_cast<O *>(base) + k);
}

template <typename S, typename O>
__global__ void __launch_bounds__(kCoupBlock)
coupling_kernel(const S *__restrict__ I, const CoupDir *__restrict__ dir, CoupArgs a) {
  using Tr = StoreTraits<S>;
  const int64_t cell = (int64_t)blockIdx.x * kCoupBlock + threadIdx.x;
  if (cell >= a.ncell) return;
  const int64_t nc = a.ncell;
  // m: E, F^x, F^y, F^z, P^xx, P^xy, P^xz, P^yy, P^yz, P^zz
  double m[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) m[k] = 0.0;
  double Ec = 0.0;   // equilibrium-shifted storage: the cell's stored E
  if constexpr (Tr::kShifted)
    Ec = (double)reinterpret_cast<const float *>(reinterpret_cast<const char *>(I) +
                                                 a.e_off)[cell];
  auto add = [&](const CoupDir &d, double v) {
    if (Tr::kReduced) v *= d.s;
    if constexpr (Tr::kShifted) v = fma(d.w, Ec, v);
    m[0] += v;
#pragma unroll
    for (int k = 0; k < 3; ++k) m[1 + k] = fma(d.n[k], v, m[1 + k]);
#pragma unroll
    for (int k = 0; k < 6; ++k) m[4 + k] = fma(d.nn[k], v, m[4 + k]);
  };
  const S *p = I + cell;
  int i = 0;
  for (; i + kCoupUnroll <= a.ndir; i += kCoupUnroll) {
    double v[kCoupUnroll];
#pragma unroll
    for (int u = 0; u < kCoupUnroll; ++u) v[u] = (double)Tr::ld(p + (int64_t)(i + u) * nc);
#pragma unroll
    for (int u = 0; u < kCoupUnroll; ++u) add(dir[i + u], v[u]);
  }
  for (; i < a.ndir; ++i) add(dir[i], (double)Tr::ld(p + (int64_t)i * nc));

  const double E = m[0];
  const double F[3] = {m[1], m[2], m[3]};
  if (a.E) put<O>(a.E, cell, E);
  if (a.F)
#pragma unroll
    for (int k = 0; k < 3; ++k) put<O>(a.F, k * nc + cell, F[k]);
  if (a.P)
#pragma unroll
    for (int k = 0; k < 6; ++k) put<O>(a.P, k * nc + cell, m[4 + k]);
  if (!a.J && !a.H && !a.S) return;

  double v[3] = {0.0, 0.0, 0.0};
  if (a.vel)
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = (double)a.vel[k * nc + cell];
  // P v with P symmetric: rows (xx xy xz), (xy yy yz), (xz yz zz)
  const double Pv[3] = {fma(m[4], v[0], fma(m[5], v[1], m[6] * v[2])),
                        fma(m[5], v[0], fma(m[7], v[1], m[8] * v[2])),
                        fma(m[6], v[0], fma(m[8], v[1], m[9] * v[2]))};
  const double v2 = fma(v[0], v[0], fma(v[1], v[1], v[2] * v[2]));
  const double W2 = 1.0 / (1.0 - v2);
  const double W = sqrt(W2);
  const double Fv = fma(F[0], v[0], fma(F[1], v[1], F[2] * v[2]));
  const double vPv = fma(Pv[0], v[0], fma(Pv[1], v[1], Pv[2] * v[2]));
  // J = W^2 (E - 2 F.v + v.P.v)
  const double J = W2 * (E - 2.0 * Fv + vPv);
  // H_j = W^3 (F.v - E) v_j + W h_ji (F - P v)^i with h_ji X^i = X_j + W^2 v_j (v.X)
  double H[3];
  const double vX = Fv - vPv;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    H[k] = W * fma(W2 * (Fv - E), v[k], fma(W2 * v[k], vX, F[k] - Pv[k]));
  const double H0 = fma(v[0], H[0], fma(v[1], H[1], v[2] * H[2]));
  if (a.J) put<O>(a.J, cell, J);
  if (a.H) {
    put<O>(a.H, cell, H0);
#pragma unroll
    for (int k = 0; k < 3; ++k) put<O>(a.H, (1 + k) * nc + cell, H[k]);
  }
  if (a.S) {
    const double ka = a.kappa_a[cell], k0 = a.kappa_s[cell], et = a.eta[cell];
    const double kt = fma(k0, a.ks_factor, ka);
    const double G = W * fma(ka, J, -et);
    put<O>(a.S, cell, fma(kt, H0, G));
#pragma unroll
    for (int k = 0; k < 3; ++k) put<O>(a.S, (1 + k) * nc + cell, fma(kt, H[k], G * v[k]));
  }
}

template <typename S, typename O>
void launch_as(const void *I, const CoupDir *dir, const CoupArgs &a, hipStream_t s) {
  const int64_t nb = (a.ncell + kCoupBlock - 1) / kCoupBlock;
  hipLaunchKernelGGL((coupling_kernel<S, O>), dim3((unsigned)nb), dim3(kCoupBlock), 0, s,
                     static_cast<const S *>(I), dir, a);
}

}  // namespace

hipError_t launch_coupling(int storage, const void *I, const CoupDir *dir, const CoupArgs &a,
                           hipStream_t s) {
  if (a.ncell <= 0) return hipSuccess;
  switch (storage) {
    case LBRT_FP32: launch_as<float, float>(I, dir, a, s); break;
    case LBRT_FP64: launch_as<double, double>(I, dir, a, s); break;
    case LBRT_BF16: launch_as<bf16_t, float>(I, dir, a, s); break;
    case LBRT_FP16: launch_as<f16_t, float>(I, dir, a, s); break;
    case LBRT_BF16_SHIFTED: launch_as<bf16s_t, float>(I, dir, a, s); break;
    default: launch_as<f16s_t, float>(I, dir, a, s); break;
  }
  return hipGetLastError();
}

}  // namespace lbrt
