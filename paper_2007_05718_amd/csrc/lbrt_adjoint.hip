// Adjoint of one stream-and-collide step: the reverse-mode sweep of a run
// that accumulates the energy detected on a face.
//
// With the forward step I' = C(S I) (S the trilinear pull of eq. (interp),
// C the implicit collision; a static fluid is the case v = 0 of the
// mixed-frame collision of App. B), the adjoint state and the coefficient
// gradients obey
//   nu      = (dC/dI*)^T lambda',          (per cell, N directions)
//   lambda  = d + S^T nu,                  (S^T: the pull from downwind cells)
//   g_k    += (dC/dk)^T lambda'            for k = kappa_a, kappa_s, eta,
// d being the detector weights of the face (the fraction dt |n^a| / dx of a
// population that leaves through it, on the face's cells).
//
// Per cell, with D_i = 1 - v.n_i, a_i = 1/(1 + dt W D_i (ka + ks)),
// c_i = dt w_i / (W^3 D_i^3), B = (dt/W) sum w_i a_i / D_i and
// J = (W^2 sum D_i^2 a_i I*_i + eta B) / (1 - ks B), the collision is
// I'_i = a_i I*_i + a_i c_i (eta + ks J).  With G = sum_i lambda'_i a_i c_i:
//   nu_i   = a_i (lambda'_i + ks W^2 D_i^2 G / (1 - ks B)),
//   g_eta += G / (1 - ks B),
//   g_ka  += -dt W sum_i lambda'_i a_i D_i I'_i + ks G dJ/dka,
//   g_ks  += -dt W sum_i lambda'_i a_i D_i I'_i + G (J + ks dJ/dks),
//   dJ/dka = (dA + eta dB + J ks dB) / (1 - ks B),
//   dJ/dks = (dA + eta dB + J (ks dB + B)) / (1 - ks B),
//   dA = -dt W^3 sum D_i^3 a_i^2 I*_i,  dB = -dt^2 sum w_i a_i^2.
//
// Two kernels: adj_collide (one thread per cell, runtime loops over the
// directions; the nu buffer first holds I* between its passes) and
// adj_transpose (one thread per population).  This is the backward sweep,
// run once per forward step of a differentiated run; it is written for
// clarity and coalesced access, not fused like the forward step.
#include "lbrt_step_kernel.h"

namespace lbrt {
namespace {

// I*_i at cell (x, y, z): the 8-tap pull with the forward step's boundary
// rules (periodic wrap; a point outside along exactly one axis takes that
// face's inflow ghost value for the slot, if any; vacuum otherwise).
template <typename T>
__device__ T pull8(const T *__restrict__ I, const DirTab<T> &d, const float *const *ghost,
                   int x, int y, int z, const KParams &p) {
  const int n3[3] = {p.nx, p.ny, p.nz};
  T acc = T(0);
  for (int b = 0; b < 8; ++b) {
    const T wt = d.tw[b];
    if (wt == T(0)) continue;
    int c[3] = {x - (b & 1) * d.s[0], y - ((b >> 1) & 1) * d.s[1], z - (b >> 2) * d.s[2]};
    int nout = 0, oa = -1;
    for (int a = 0; a < 3; ++a) {
      if (p.periodic[a]) c[a] = wrap(c[a], n3[a]);
      if ((unsigned)c[a] >= (unsigned)n3[a]) {
        ++nout;
        oa = a;
      }
    }
    T v = T(0);
    if (nout == 0) {
      v = I[d.plane_el + ((int64_t)c[2] * p.ny + c[1]) * p.nx + c[0]];
    } else if (nout == 1 && ghost[oa] != nullptr) {
      // face layouts: x faces [z][y], y faces [z][x], z faces [y][x]
      const int64_t gi = oa == 0 ? (int64_t)c[2] * p.ny + c[1]
                                 : (oa == 1 ? (int64_t)c[2] * p.nx + c[0]
                                            : (int64_t)c[1] * p.nx + c[0]);
      v = (T)ghost[oa][gi];
    }
    acc = fma(wt, v, acc);
  }
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
adj_collide_kernel(const T *__restrict__ I, const T *__restrict__ lam, T *__restrict__ nu,
                   T *__restrict__ g_ka, T *__restrict__ g_ks, T *__restrict__ g_eta,
                   const float *__restrict__ ka, const float *__restrict__ ks,
                   const float *__restrict__ eta, const float *__restrict__ vel,
                   const DirTab<T> *__restrict__ tab, const KParams p,
                   const InflowArgs *__restrict__ inflow) {
  const int64_t cell = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= p.ncell) return;
  const int x = (int)(cell % p.nx);
  const int y = (int)((cell / p.nx) % p.ny);
  const int z = (int)(cell / ((int64_t)p.nx * p.ny));
  const T dt = (T)p.dt;
  const T kat = (T)ka[cell], kst = (T)ks[cell], et = (T)eta[cell];
  T vx = T(0), vy = T(0), vz = T(0);
  if (vel != nullptr) {
    vx = (T)vel[cell];
    vy = (T)vel[p.ncell + cell];
    vz = (T)vel[2 * p.ncell + cell];
  }
  const T W = T(1) / sqrt(T(1) - (vx * vx + vy * vy + vz * vz));
  const T kt = kat + kst;
  // pass 1: I*_i (kept in nu), and the sums of A, B, dA, dB
  T sA = T(0), sB = T(0), sdA = T(0), sdB = T(0);
  for (int k = 0; k < p.ndir; ++k) {
    const DirTab<T> &d = tab[k];
    const T Is = pull8<T>(I, d, inflow->ghost[k], x, y, z, p);
    nu[d.plane_el + cell] = Is;
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = T(1) / (T(1) + dt * W * D * kt);
    sA = fma(D * D * a, Is, sA);
    sB += d.w * a / D;
    sdA = fma(D * D * D * a * a, Is, sdA);
    sdB += d.w * a * a;
  }
  const T A = W * W * sA;
  const T B = dt / W * sB;
  const T den = T(1) - kst * B;
  const T J = (A + et * B) / den;
  const T W3 = W * W * W;
  // pass 2: G = sum lambda'_i a_i c_i, and sum lambda'_i a_i D_i I'_i
  T G = T(0), sM = T(0);
  for (int k = 0; k < p.ndir; ++k) {
    const DirTab<T> &d = tab[k];
    const T Is = nu[d.plane_el + cell];
    const T mu = lam[d.plane_el + cell];
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = T(1) / (T(1) + dt * W * D * kt);
    const T c = dt * d.w / (W3 * D * D * D);
    const T Ip = a * (Is + c * (et + kst * J));
    G = fma(mu, a * c, G);
    sM = fma(mu * a * D, Ip, sM);
  }
  const T dA = -dt * W3 * sdA;
  const T dB = -dt * dt * sdB;
  const T dJa = (dA + et * dB + J * kst * dB) / den;
  const T dJs = (dA + et * dB + J * (kst * dB + B)) / den;
  g_ka[cell] += -dt * W * sM + kst * G * dJa;
  g_ks[cell] += -dt * W * sM + G * (J + kst * dJs);
  g_eta[cell] += G / den;
  // pass 3: nu_i
  const T h = kst * W * W * G / den;
  for (int k = 0; k < p.ndir; ++k) {
    const DirTab<T> &d = tab[k];
    const T mu = lam[d.plane_el + cell];
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = T(1) / (T(1) + dt * W * D * kt);
    nu[d.plane_el + cell] = a * fma(h, D * D, mu);
  }
}

// lambda_i(r) = d_i(r) + sum_b w_b nu_i(r + b.s_i): the transpose of the pull
// (sources outside the box are ghosts and get nothing; periodic axes wrap).
template <typename T>
__global__ void __launch_bounds__(kBlock)
adj_transpose_kernel(const T *__restrict__ nu, T *__restrict__ lam,
                     const DirTab<T> *__restrict__ tab, const KParams p, int face) {
  const int64_t total = p.ncell * p.ndir;
  const int n3[3] = {p.nx, p.ny, p.nz};
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kBlock) {
    const int k = (int)(e / p.ncell);
    const int64_t cell = e - (int64_t)k * p.ncell;
    const DirTab<T> &d = tab[k];
    const int r[3] = {(int)(cell % p.nx), (int)((cell / p.nx) % p.ny),
                      (int)(cell / ((int64_t)p.nx * p.ny))};
    T acc = T(0);
    for (int b = 0; b < 8; ++b) {
      const T wt = d.tw[b];
      if (wt == T(0)) continue;
      int c[3] = {r[0] + (b & 1) * d.s[0], r[1] + ((b >> 1) & 1) * d.s[1],
                  r[2] + (b >> 2) * d.s[2]};
      bool in = true;
      for (int a = 0; a < 3; ++a) {
        if (p.periodic[a]) c[a] = wrap(c[a], n3[a]);
        in = in && (unsigned)c[a] < (unsigned)n3[a];
      }
      if (in) acc = fma(wt, nu[d.plane_el + ((int64_t)c[2] * p.ny + c[1]) * p.nx + c[0]], acc);
    }
    if (face >= 0) {
      // detector: the part of the population that leaves through the face
      const int a = face >> 1;
      const bool hi = (face & 1) != 0;
      const bool on = hi ? r[a] == n3[a] - 1 : r[a] == 0;
      const bool leaves = hi ? d.s[a] > 0 : d.s[a] < 0;
      if (on && leaves && !p.periodic[a]) acc += d.delta[a];
    }
    lam[d.plane_el + cell] = acc;
  }
}

}  // namespace

hipError_t launch_adjoint(int storage, const void *I, const void *lam_next, void *lam_out,
                          void *nu, int face, void *g_ka, void *g_ks, void *g_eta,
                          const float *ka, const float *ks, const float *eta, const float *vel,
                          const void *tab, const KParams &p, const InflowArgs *inflow,
                          hipStream_t s) {
  const int nb = (int)((p.ncell + kBlock - 1) / kBlock);
  const int64_t tot = p.ncell * p.ndir;
  const int nb2 = (int)std::min<int64_t>((tot + kBlock - 1) / kBlock, 65536);
  if (storage == LBRT_FP64) {
    using T = double;
    hipLaunchKernelGGL(adj_collide_kernel<T>, dim3(nb), dim3(kBlock), 0, s,
                       static_cast<const T *>(I), static_cast<const T *>(lam_next),
                       static_cast<T *>(nu), static_cast<T *>(g_ka), static_cast<T *>(g_ks),
                       static_cast<T *>(g_eta), ka, ks, eta, vel,
                       static_cast<const DirTab<T> *>(tab), p, inflow);
    hipLaunchKernelGGL(adj_transpose_kernel<T>, dim3(nb2), dim3(kBlock), 0, s,
                       static_cast<const T *>(nu), static_cast<T *>(lam_out),
                       static_cast<const DirTab<T> *>(tab), p, face);
  } else {
    using T = float;
    hipLaunchKernelGGL(adj_collide_kernel<T>, dim3(nb), dim3(kBlock), 0, s,
                       static_cast<const T *>(I), static_cast<const T *>(lam_next),
                       static_cast<T *>(nu), static_cast<T *>(g_ka), static_cast<T *>(g_ks),
                       static_cast<T *>(g_eta), ka, ks, eta, vel,
                       static_cast<const DirTab<T> *>(tab), p, inflow);
    hipLaunchKernelGGL(adj_transpose_kernel<T>, dim3(nb2), dim3(kBlock), 0, s,
                       static_cast<const T *>(nu), static_cast<T *>(lam_out),
                       static_cast<const DirTab<T> *>(tab), p, face);
  }
  return hipGetLastError();
}

}  // namespace lbrt
