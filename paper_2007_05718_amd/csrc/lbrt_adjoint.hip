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
// d being the detector weights of the face: on the face's cells, the
// fraction of a population that the forward step books as outflux through
// that face (dt |n^a| / dx, reduced on edges and corners where part of it
// is booked on an earlier face in the order x, y, z).
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
// Three launches: adj_pull<false> computes I* = S I into the nu buffer (the
// forward pull with its boundary rules); adj_collide (one thread per cell,
// two passes over the directions) turns it into nu and adds the gradients;
// adj_pull<true> computes lambda = d + S^T nu.  S^T is the same pull with
// the shift signs reversed and no ghosts (a source outside the box gets
// nothing back).  The pulls march one direction per block through z with
// the separable form of the trilinear weights, like the forward step, so a
// plane costs four row loads per direction instead of eight gathers.
#include "lbrt_step_kernel.h"

namespace lbrt {
namespace {

constexpr int kPullRows = 4;    // rows (waves) per block of adj_pull
constexpr int kPullZlen = 32;   // z planes marched per block

// One direction per block (blockIdx.y, processing order), a 64 x kPullRows
// tile of cells per block, marched through kPullZlen planes.  REV = false:
// out = S in (the forward pull: periodic wrap; a tap outside the box along
// exactly one axis takes that face's inflow ghost value, if any, else 0).
// REV = true: out = d + S^T in (shift signs reversed, taps outside give 0,
// d = the detector weights of `face` on its cells, face < 0 for none).
template <typename T, bool REV>
__global__ void __launch_bounds__(64 * kPullRows)
adj_pull_kernel(const T *__restrict__ in, T *__restrict__ out, const DirTab<T> *__restrict__ tab,
                const KParams p, const InflowArgs *__restrict__ inflow, int face) {
  const int k = blockIdx.y;
  const DirTab<T> &d = tab[k];
  const int ntx = (p.nx + 63) >> 6, nty = (p.ny + kPullRows - 1) / kPullRows;
  const int bx = blockIdx.x % ntx, r = blockIdx.x / ntx;
  const int by = r % nty, bz = r / nty;
  const int x = bx * 64 + (threadIdx.x & 63);
  const int y = by * kPullRows + (threadIdx.x >> 6);
  const int zb = bz * kPullZlen, ze = min(p.nz, zb + kPullZlen);
  if (x >= p.nx || y >= p.ny) return;
  const int sg = REV ? -1 : 1;
  const int sx = sg * d.s[0], sy = sg * d.s[1], sz = sg * d.s[2];
  const int n3[3] = {p.nx, p.ny, p.nz};
  const float *const *ghost = REV ? nullptr : inflow->ghost[k];
  const int64_t pc = (int64_t)p.nx * p.ny;
  const T *src = in + d.plane_el;

  // Tap (cx, cy, cz) after periodic wrapping: its element index in the
  // direction's plane when inside the box, else the axis it leaves along
  // (oa) and how many axes it leaves along (nout).
  struct Tap {
    int c[3];
    int nout, oa;
  };
  auto locate = [&](int cx, int cy, int cz) {
    Tap t{{cx, cy, cz}, 0, 0};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (p.periodic[a]) t.c[a] = wrap(t.c[a], n3[a]);
      if ((unsigned)t.c[a] >= (unsigned)n3[a]) {
        ++t.nout;
        t.oa = a;
      }
    }
    return t;
  };
  // A tap outside the box: the face's inflow ghost value when it leaves
  // along exactly one axis and that face has a ghost plane, else 0.
  auto outside = [&](const Tap &t) -> T {
    if (REV || t.nout > 1 || ghost[t.oa] == nullptr) return T(0);
    // face layouts: x faces [z][y], y faces [z][x], z faces [y][x]
    const int64_t gi = t.oa == 0 ? (int64_t)t.c[2] * p.ny + t.c[1]
                                 : (t.oa == 1 ? (int64_t)t.c[2] * p.nx + t.c[0]
                                              : (int64_t)t.c[1] * p.nx + t.c[0]);
    return (T)gload(ghost[t.oa], gi);
  };
  // plane value P(zl): the x/y interpolation of the four taps of plane zl.
  // The four in-box loads go out together (a tap outside the box reads
  // element 0 and is replaced), so that a plane costs one wait, not four.
  auto plane = [&](int zl) -> T {
    const Tap t[4] = {locate(x, y, zl), locate(x - sx, y, zl), locate(x, y - sy, zl),
                      locate(x - sx, y - sy, zl)};
    T v[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t i = t[b].nout == 0
                            ? (int64_t)t[b].c[2] * pc + (int64_t)t[b].c[1] * p.nx + t[b].c[0]
                            : 0;
      v[b] = src[i];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (t[b].nout != 0) v[b] = outside(t[b]);
    return interp4(d, v[0], v[1], v[2], v[3]);
  };
  const T dz = d.delta[2], dz1 = T(1) - d.delta[2];
  // I*(z) = (1 - dz) P(z) + dz P(z - sz), marching up in z with one carried
  // plane value: P(z - 1) when sz > 0, P(z) when sz < 0
  T carry = sz > 0 ? plane(zb - 1) : (sz < 0 ? plane(zb) : T(0));
  // detector: the cells on `face` for a direction that leaves through it.
  // The weight is the fraction of the population that the forward step
  // books on that face (the step kernels' rule): dt |n^a| / dx, times
  // (1 - dt |n^b| / dx) for each earlier axis b (order x, y, z) whose
  // non-periodic face the cell also leaves through.
  bool det = false;
  T dw = T(0);
  const int c3[2] = {x, y};
  if (REV && face >= 0) {
    const int a = face >> 1;
    const bool hi = (face & 1) != 0;
    const bool leaves = hi ? d.s[a] > 0 : d.s[a] < 0;
    det = leaves && !p.periodic[a];
    dw = d.delta[a];
    // the earlier axes (x, and y for a z face) are fixed per thread
    for (int b = 0; b < a && b < 2; ++b) {
      const bool out_b = !p.periodic[b] && ((d.s[b] > 0 && c3[b] == n3[b] - 1) ||
                                            (d.s[b] < 0 && c3[b] == 0));
      if (out_b) dw *= T(1) - d.delta[b];
    }
  }
  for (int z = zb; z < ze; ++z) {
    T v;
    if (sz > 0) {
      const T pz = plane(z);
      v = fma(dz, carry, dz1 * pz);
      carry = pz;
    } else if (sz < 0) {
      const T pn = plane(z + 1);
      v = fma(dz, pn, dz1 * carry);
      carry = pn;
    } else {
      v = plane(z);
    }
    if (REV && det) {
      const int a = face >> 1;
      const int ra = a == 0 ? x : (a == 1 ? y : z);
      if (ra == ((face & 1) ? n3[a] - 1 : 0)) v += dw;
    }
    out[d.plane_el + (int64_t)z * pc + (int64_t)y * p.nx + x] = v;
  }
}

// Per cell: nu = (dC/dI*)^T lambda' from I* (in nu on entry) and lambda',
// and the coefficient gradients.  Pass 1 forms every sum at once: the part
// of sum_i lambda'_i a_i D_i I'_i that depends on J is split off
// (I'_i = a_i (I*_i + c_i (eta + ks J))), so J is not needed until after
// the pass.  Pass 2 writes nu over I*.
template <typename T>
__global__ void __launch_bounds__(kBlock)
adj_collide_kernel(const T *__restrict__ lam, T *__restrict__ nu, T *__restrict__ g_ka,
                   T *__restrict__ g_ks, T *__restrict__ g_eta, const float *__restrict__ ka,
                   const float *__restrict__ ks, const float *__restrict__ eta,
                   const float *__restrict__ vel, const DirTab<T> *__restrict__ tab,
                   const KParams p) {
  const int64_t cell = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (cell >= p.ncell) return;
  const T dt = (T)p.dt;
  const T kat = (T)ka[cell], kst = (T)ks[cell], et = (T)eta[cell];
  T vx = T(0), vy = T(0), vz = T(0);
  if (vel != nullptr) {
    vx = (T)vel[cell];
    vy = (T)vel[p.ncell + cell];
    vz = (T)vel[2 * p.ncell + cell];
  }
  const T W = div_fast(T(1), sqrt(T(1) - (vx * vx + vy * vy + vz * vz)));
  const T W3 = W * W * W;
  const T dtWk = dt * W * (kat + kst);
  T sA = T(0), sB = T(0), sdA = T(0), sdB = T(0), G = T(0), sM1 = T(0), sM2 = T(0);
  for (int k = 0; k < p.ndir; ++k) {
    const DirTab<T> &d = tab[k];
    const T Is = nu[d.plane_el + cell];
    const T mu = lam[d.plane_el + cell];
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T iD = div_fast(T(1), D);
    const T a = div_fast(T(1), fma(dtWk, D, T(1)));
    const T c = dt * d.w * iD * iD * iD / W3;
    sA = fma(D * D * a, Is, sA);
    sB = fma(d.w * a, iD, sB);
    sdA = fma(D * D * D * a * a, Is, sdA);
    sdB = fma(d.w * a, a, sdB);
    G = fma(mu, a * c, G);
    const T mad = mu * a * a * D;
    sM1 = fma(mad, Is, sM1);
    sM2 = fma(mad, c, sM2);
  }
  const T A = W * W * sA;
  const T B = dt / W * sB;
  const T den = T(1) - kst * B;
  const T J = div_fast(A + et * B, den);
  const T sM = fma(et + kst * J, sM2, sM1);
  const T dA = -dt * W3 * sdA;
  const T dB = -dt * dt * sdB;
  const T dJa = div_fast(dA + et * dB + J * kst * dB, den);
  const T dJs = div_fast(dA + et * dB + J * (kst * dB + B), den);
  g_ka[cell] += -dt * W * sM + kst * G * dJa;
  g_ks[cell] += -dt * W * sM + G * (J + kst * dJs);
  g_eta[cell] += div_fast(G, den);
  const T h = div_fast(kst * W * W * G, den);
  for (int k = 0; k < p.ndir; ++k) {
    const DirTab<T> &d = tab[k];
    const T mu = lam[d.plane_el + cell];
    const T D = T(1) - (vx * d.n[0] + vy * d.n[1] + vz * d.n[2]);
    const T a = div_fast(T(1), fma(dtWk, D, T(1)));
    nu[d.plane_el + cell] = a * fma(h, D * D, mu);
  }
}

template <typename T>
void launch_adjoint_t(const void *I, const void *lam_next, void *lam_out, void *nu, int face,
                      void *g_ka, void *g_ks, void *g_eta, const float *ka, const float *ks,
                      const float *eta, const float *vel, const void *tab, const KParams &p,
                      const InflowArgs *inflow, hipStream_t s) {
  const int nc = (int)((p.ncell + kBlock - 1) / kBlock);
  const int ntx = (p.nx + 63) >> 6, nty = (p.ny + kPullRows - 1) / kPullRows;
  const int nzr = (p.nz + kPullZlen - 1) / kPullZlen;
  const dim3 pg((unsigned)(ntx * nty * nzr), (unsigned)p.ndir);
  const DirTab<T> *t = static_cast<const DirTab<T> *>(tab);
  hipLaunchKernelGGL((adj_pull_kernel<T, false>), pg, dim3(64 * kPullRows), 0, s,
                     static_cast<const T *>(I), static_cast<T *>(nu), t, p, inflow, -1);
  hipLaunchKernelGGL(adj_collide_kernel<T>, dim3(nc), dim3(kBlock), 0, s,
                     static_cast<const T *>(lam_next), static_cast<T *>(nu),
                     static_cast<T *>(g_ka), static_cast<T *>(g_ks), static_cast<T *>(g_eta),
                     ka, ks, eta, vel, t, p);
  hipLaunchKernelGGL((adj_pull_kernel<T, true>), pg, dim3(64 * kPullRows), 0, s,
                     static_cast<const T *>(nu), static_cast<T *>(lam_out), t, p, inflow, face);
}

}  // namespace

hipError_t launch_adjoint(int storage, const void *I, const void *lam_next, void *lam_out,
                          void *nu, int face, void *g_ka, void *g_ks, void *g_eta,
                          const float *ka, const float *ks, const float *eta, const float *vel,
                          const void *tab, const KParams &p, const InflowArgs *inflow,
                          hipStream_t s) {
  if (storage == LBRT_FP64)
    launch_adjoint_t<double>(I, lam_next, lam_out, nu, face, g_ka, g_ks, g_eta, ka, ks, eta,
                             vel, tab, p, inflow, s);
  else
    launch_adjoint_t<float>(I, lam_next, lam_out, nu, face, g_ka, g_ks, g_eta, ka, ks, eta,
                            vel, tab, p, inflow, s);
  return hipGetLastError();
}

}  // namespace lbrt
