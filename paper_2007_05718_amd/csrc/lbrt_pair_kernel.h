// The fused step on interior tiles with two adjacent x cells per lane.
//
// A block owns a row segment of 128 cells (64 lanes, cells x0 + 2l and
// x0 + 2l + 1 on lane l) and marches it through a range of z planes, like
// the main kernel of lbrt_step_kernel.h, with its NW waves splitting the
// direction slots.  Each slot's constants, addresses and loads then serve two
// cells: a row load is one dword holding both cells' BF16 or FP16 values, so
// a plane costs four loads per direction for two cells and one store.
//
// The x-shifted pair of a row, cells (x - sx, x + 1 - sx), comes from the
// neighbouring pair (the one before it for sx > 0, after it otherwise; for
// sx = 0 its weight is 0), an aligned load like the own pair, by one
// v_perm_b32 of the two dwords with the slot's byte selector.
//
// Equilibrium-shifted 16-bit storage takes it too: the block stages the E
// cells its slots' taps read (three rows of 130 cells per plane) in LDS, a
// slot pulls E with the populations' weights from there, carries the
// population's plane value s_i P + w_i P_E, and stores the deviation from
// w_i E' and E' itself (the same arithmetic as the other paths).
//
// Only the 16-bit forms take this path.  With FP32 storage a two-cell lane
// holds twice the bytes per slot in flight, so under the same register
// budget it keeps half as many slots ahead per cell and waits longer on its
// loads than the one-cell main kernel (built under the 128-VGPR cap of two
// blocks per CU it spills even with two slots ahead); the main kernel
// serves FP32.
// The slot constants come from compact records (PairTab, PairColl), each
// read with one wide scalar load per plane.
//
// The tiles start at x = 128 k, so a wave's row loads and stores are whole
// cache lines; they compute rows [1, ny - 1), whose y halo is inside the box.
// With non-periodic x faces they compute every cell of the row: the first
// and last pair are face pairs, whose neighbouring pair for sx > 0 (first)
// or sx < 0 (last) is a ghost: the lane loads its own pair in its place and
// zeroes it; an inflow ghost plane on the face is added afterwards
// (x_ghost_correction, as on the other paths).  The zeroing is two ANDs per
// slot on every tile, with a per-lane mask picked by the slot's sign (a
// second copy of the slot loop for the face tiles only would run the kernel
// out of scalar registers; per-slot selects on the face flags cost three
// more VALU instructions per slot, 1-2 % of the step).  The x-face outflux of
// the face cells is booked after each plane from their own values parked in
// LDS, one slot per lane.  With periodic x the tiles compute
// x in [2, nx - 2) and the columns x < 2, x >= nx - 2 are tiles of the
// general (checked) path, like the face rows.  nx is even, so every pair
// starts at an even cell index and its loads and stores are aligned.
// (Reading the face columns on the general path instead would fetch a whole
// cache line of a row for each pair: for 16-bit storage that path took a
// third of the step's time at 256^3.)
//
// Per plane:
//   stream   the wave's slots for both cells (P from 4 row loads, issued a few
//            slots ahead; I* from P and the carried plane value);
//   moments  per-wave partial E*, F* of the 128 cells into LDS; barrier;
//   combine  the 512 sums (4 moments x 128 cells) are split over the block:
//            each lane forms one or two of them over the waves (a fixed
//            pairwise order, the general path's), then the collision's E or
//            F part for that cell (coef_E / coef_F), writes E or F, and puts
//            c, alpha (and beta) in LDS; barrier;
//   collide  every wave reads its cells' c, alpha (beta) and writes the new
//            populations of its slots, one store per slot for both cells.
// A cell gives the same bits here as on the general path: the same per-slot
// arithmetic, the same summation order, the same collision functions and the
// same random bits for stochastic rounding.
#pragma once

namespace lbrt {

typedef float f32x2 __attribute__((ext_vector_type(2)));

template <typename S> struct PairIO;

template <typename S> struct PairIO16 {
  using R = uint32_t;
  static constexpr uint32_t kShift = 4;   // byte offset of the neighbouring pair
  __device__ static R ld(const char *b, uint32_t off) {
    return *reinterpret_cast<const uint32_t *>(b + off);
  }
  // the x-shifted pair (nb.hi, own.lo) for sx > 0, else (own.hi, nb.lo)
  __device__ static R shifted(R own, R nb, bool pos) {
    return __builtin_amdgcn_perm(own, nb, pos ? 0x05040302u : 0x01000706u);
  }
};

template <> struct PairIO<bf16_t> : PairIO16<bf16_t> {
  __device__ static float lo(R v) { return __uint_as_float(v << 16); }
  __device__ static float hi(R v) { return __uint_as_float(v & 0xffff0000u); }
  // the shifted cells as FP32 bit patterns in one v_perm_b32 each: the BF16
  // half into the high 16 bits, zeros (byte selector 0x0c) below
  __device__ static float shifted_lo(R own, R nb, bool pos) {
    return __uint_as_float(__builtin_amdgcn_perm(own, nb, pos ? 0x03020c0cu : 0x07060c0cu));
  }
  __device__ static float shifted_hi(R own, R nb, bool pos) {
    return __uint_as_float(__builtin_amdgcn_perm(own, nb, pos ? 0x05040c0cu : 0x01000c0cu));
  }
  __device__ static void st(char *b, uint32_t off, float a, float c, uint32_t ra, uint32_t rc,
                            bool sr) {
    uint32_t w;
    if (sr) {
      s16x2 h = __builtin_amdgcn_cvt_sr_bf16_f32(s16x2{0, 0}, a, ra, false);
      h = __builtin_amdgcn_cvt_sr_bf16_f32(h, c, rc, true);
      w = __builtin_bit_cast(uint32_t, h);
    } else {
      typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
      w = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, c}, bf16x2));
    }
    __builtin_nontemporal_store(w, reinterpret_cast<uint32_t *>(b + off));
  }
};

template <> struct PairIO<f16_t> : PairIO16<f16_t> {
  __device__ static float lo(R v) {
    return (float)__builtin_bit_cast(f16x2, v).x;
  }
  __device__ static float hi(R v) {
    return (float)__builtin_bit_cast(f16x2, v).y;
  }
  __device__ static float shifted_lo(R own, R nb, bool pos) { return lo(shifted(own, nb, pos)); }
  __device__ static float shifted_hi(R own, R nb, bool pos) { return hi(shifted(own, nb, pos)); }
  __device__ static void st(char *b, uint32_t off, float a, float c, uint32_t ra, uint32_t rc,
                            bool sr) {
    f16x2 h;
    if (sr) {
      h = __builtin_amdgcn_cvt_sr_f16_f32(f16x2{0, 0}, a, ra, false);
      h = __builtin_amdgcn_cvt_sr_f16_f32(h, c, rc, true);
    } else {
      h = __builtin_convertvector(f32x2{a, c}, f16x2);
    }
    __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, h),
                                reinterpret_cast<uint32_t *>(b + off));
  }
};

// Equilibrium-shifted storage: the stored deviations are BF16 / FP16 pairs
// like the plain forms'.
template <> struct PairIO<bf16s_t> : PairIO<bf16_t> {};
template <> struct PairIO<f16s_t> : PairIO<f16_t> {};

// Compiled combinations: static fluid, BF16 / FP16 storage (plain or
// equilibrium-shifted), the 56- and 112-slot buckets.
template <typename S, int NB, bool MOVING>
constexpr bool pair_kernel_exists() {
  return !MOVING && sizeof(S) == 2 && (NB == 56 || NB == 112);
}

// Equilibrium-shifted storage: a block stages the E cells that its slots'
// taps read (rows y - 1 .. y + 1, columns x0 - 1 .. x0 + 128) in LDS per
// plane; staged cell (r, c) sits at element 1 + r kPairSRow + c, so that a
// lane's own pair (c = 2l + 1, 2l + 2) is one aligned 8-byte read.
constexpr int kPairSRow = 130;
constexpr int kPairSPos = 3 * kPairSRow;
constexpr int kPairSBuf = kPairSPos + 2;

// Slots whose four row loads (4 VGPRs) are in flight ahead of the slot being
// interpolated.  Two 8-wave blocks per CU need at most 128 VGPRs: BF16 keeps
// 4 ahead (127 VGPRs; 3 ahead measured 3 % slower); FP16, whose conversions
// take a few more registers, 3 (4 needs 129: one block per CU, 1.5x the
// time; bounded to 128 it spills and is 7 % slower than 3 ahead).  Shifted
// storage, whose E taps and staging take more registers, is bounded to 128
// VGPRs (below) and keeps 3 ahead with 112 slots (28 bytes of spill per
// lane, 3.5 % faster than 2 ahead), 2 with 56 (3 was 2 % slower).
template <typename S, int NB>
constexpr int pair_pf_depth(int m) {
  const int d = StoreTraits<S>::kShifted ? (NB >= 112 ? 3 : 2)
                                         : (std::is_same_v<S, f16_t> ? 3 : 4);
  return m < d ? m : d;
}

// Waves per SIMD the pair kernel is bounded for (a VGPR cap of 512 / w).
// The shifted kernels exceed 128 VGPRs unbounded (133 with 56 slots and 2
// ahead, where the bound costs 12 bytes of spill and runs 5 % faster than
// three waves per SIMD).  The others fit 128 unbounded (a bound makes the
// allocator spill).
template <typename S, int NB>
constexpr int pair_waves_per_simd() {
  return StoreTraits<S>::kShifted ? 4 : waves_per_simd<S>(NB);
}

// Plane value from four taps with the slot's per-axis weights: the same
// rounding order as interp4.
__device__ __forceinline__ float interp4w(const PairTab &d, float a, float a1, float b,
                                          float b1) {
  return lerp2(d.wy0, d.wy1, lerp2(d.wx0, d.wx1, a, a1), lerp2(d.wx0, d.wx1, b, b1));
}

// New population of one direction of a cell (collide_one with a PairColl).
__device__ __forceinline__ float collide_pair(const PairColl &d, float c, float alpha, float b0,
                                              float b1, float b2, float Is, bool lamzero) {
  if (lamzero) return fma(c, Is, d.w * alpha);
  const float nb = fma(d.n2, b2, fma(d.n1, b1, fma(d.n0, b0, alpha)));
  return fma(c, Is, d.w * nb);
}

template <typename S, int NB, int NW = waves_for(NB)>
__device__ __forceinline__ void
march_pair(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
           const float *__restrict__ ks, const float *__restrict__ eta,
           const PairTab *__restrict__ tab, const PairColl *__restrict__ ctab,
           const DirTab<float> *__restrict__ dtab, const InflowArgs *__restrict__ inflow,
           const KParams &p, float *__restrict__ Eout, float *__restrict__ Fout,
           double *__restrict__ partials, int x0, int y, int zb, int ze) {
  using IO = PairIO<S>;
  using R = typename IO::R;
  using T = float;
  constexpr int SZ = (int)sizeof(S);
  constexpr int M = NB / NW;
  constexpr int NC = 128;                       // cells of a tile
  constexpr int RI = 4 * NC / (64 * NW);        // combine items per lane
  static_assert(4 * NC % (64 * NW) == 0, "combine items must split evenly");
  constexpr int D = pair_pf_depth<S, NB>(M);

  const int nx = p.nx, nz = p.nz;
  const int64_t pc = (int64_t)nx * p.ny;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int perz = p.periodic[2];
  const int xend = p.pair_xend;
  const T dt = (T)p.dt;
  const bool diag = (p.flags & KF_DIAG) != 0;
  const bool stoch = (p.flags & KF_STOCH) != 0;
  // Equilibrium-shifted storage: the states' FP32 E arrays (byte offset e_off)
  constexpr bool SH = StoreTraits<S>::kShifted;
  const char *const ein_bytes = reinterpret_cast<const char *>(Iin) + (SH ? p.e_off : 0);
  char *const eout_bytes = reinterpret_cast<char *>(Iout) + (SH ? p.e_off : 0);
  // staged E cells, three plane buffers (see the staging below)
  __shared__ __attribute__((aligned(16))) float estage[SH ? 3 : 1][SH ? kPairSBuf : 2];

  // stream lanes: cells (x, x + 1), stored when inside [pair_x0, pair_xend);
  // a lane beyond the row reads the last pair
  int x = x0 + 2 * lane;
  const bool valid = x >= p.pair_x0 && x < xend;
  if (x >= xend) x = xend - 2;
  const uint32_t o0 = (uint32_t)(x + nx * y) * (uint32_t)SZ;
  // face pairs of a non-periodic x axis (pair_x0 = 0, pair_xend = nx then)
  const int perx = p.periodic[0];
  const bool lox = valid && !perx && x == 0;
  const bool hix = valid && !perx && x + 2 == nx;
  const bool xface_tile = !perx && (x0 == 0 || x0 + NC >= nx);
  // combine lanes: cell cc of the tile
  const int cc = (q & 1) * 64 + lane;
  int xc = x0 + cc;
  const bool valid_c = xc >= p.pair_x0 && xc < xend;
  if (xc >= xend) xc = xend - 1;
  const uint32_t ocell = (uint32_t)(xc + nx * y);

  const PairTab *__restrict__ tb = tab + q * M;
  const char *const in_bytes = reinterpret_cast<const char *>(Iin);

  // the four row loads of slot d from the z-plane starting at byte `plane`
  // (rows y and y - sy; own and neighbouring pair)
  // The neighbouring pair's shift goes into the wave-uniform base, so the
  // loads take a scalar base plus a 32-bit lane offset: o0 for the own pair;
  // for the neighbouring pair o0 too, except on a lane whose pair is the
  // first (sx > 0) or the last (sx < 0) of its row, whose neighbouring pair
  // is outside the row: that lane reads its own pair again (its values are
  // then zeroed, or unused), so that no load leaves the row, and no load
  // leaves the state's buffer (the row before the first or after the last
  // of a plane can be outside it).
  const uint32_t onp = x == 0 ? o0 + IO::kShift : o0;
  const uint32_t onm = x + 2 == nx ? o0 - IO::kShift : o0;
  auto load4 = [&](const PairTab &d, const char *plane, R (&v)[4]) {
    const char *r0 = plane + d.plane_off;
    const char *r1 = r0 + d.row_off;
    const bool pos = (d.flags & kPairSxPos) != 0;
    const int sh = pos ? -(int)IO::kShift : (int)IO::kShift;
    const uint32_t oo = opaque_lane(o0);
    const uint32_t on = opaque_lane(pos ? onp : onm);
    v[0] = IO::ld(r0, oo);
    v[1] = IO::ld(r0 + sh, on);
    v[2] = IO::ld(r1, oo);
    v[3] = IO::ld(r1 + sh, on);
  };
  // plane values of both cells from a slot's four loads
  auto interp2 = [&](const PairTab &d, const R (&v)[4], T &Plo, T &Phi) {
    const bool pos = (d.flags & kPairSxPos) != 0;
    Plo = interp4w(d, IO::lo(v[0]), IO::shifted_lo(v[0], v[1], pos), IO::lo(v[2]),
                   IO::shifted_lo(v[2], v[3], pos));
    Phi = interp4w(d, IO::hi(v[0]), IO::shifted_hi(v[0], v[1], pos), IO::hi(v[2]),
                   IO::shifted_hi(v[2], v[3], pos));
  };
  auto plane_above = [&](int z) {
    const int za = z + 1 < nz ? z + 1 : (perz ? 0 : nz - 1);
    return (int64_t)za * pc;
  };

  // Face lanes: the neighbouring pair of a slot whose x-shifted taps lie
  // outside the box is a vacuum ghost (zeroed: its in-box load is
  // discarded).
  double fin = 0.0;
  // x-face outflux of the face cells (diagnostics).  Every lane parks its
  // own pair of each slot in LDS as the slot is streamed (one ds_write per
  // slot; booking inside the slot loop would keep more of each slot's record
  // in scalar registers than the loop has).  After the plane, lane l < M of
  // a tile holding the -x face books slot l of the face pair (lane 0), and
  // lane 32 + l of a tile holding the +x face books slot l of the pair
  // (nx - 2, nx - 1): one LDS read and one FMA per lane and plane, with the
  // slot's factor dt |n^x| / dx times the storage scale (0 unless the slot
  // leaves through that face) fixed once per block.
  __shared__ R ownx[NW][M][64];
  // per booking lane: the factor (0 on a lane that books nothing), and the
  // parked value's index in ownx times 2 plus the slot's dzn bit
  T bf = T(0), fxb = T(0);
  uint32_t bix = 0u;
  // shifted storage: the E part of the booked value (dt |n^x| / dx times w,
  // or 0) and the staged index of the face cell (row y)
  T bfE = T(0);
  int eix = 0;
  {
    const bool has_lo = diag && !perx && x0 == 0;
    const bool has_hi = diag && !perx && x0 + NC >= nx;
    const bool hi = lane >= 32;
    const int slot = lane & 31;
    if (slot < M && (hi ? has_hi : has_lo)) {
      const DirTab<T> &d = dtab[q * M + slot];
      bf = (hi ? d.s[0] > 0 : d.s[0] < 0) ? d.dxs : T(0);
      if constexpr (SH) bfE = bf != T(0) ? d.delta[0] * d.w : T(0);
      eix = 1 + kPairSRow + (hi ? nx - x0 : 1);
      const int src = hi ? (nx - 2 - x0) >> 1 : 0;
      bix = (uint32_t)(((q * M + slot) * 64 + src) * 2 + d.dzn);
    }
  }
  // (a slot that books nothing is skipped, not multiplied by 0: its parked
  // value may be unwritten LDS, e.g. a slot the prologue did not load)
  // (shifted storage: the staged E of the face cell at the booked plane is in
  // ring buffer b0 (the plane) or b1 (the plane above, dzn slots))
  auto book_face = [&](bool prologue, int lastz, int b0, int b1) {
    const int dzn = (int)(bix & 1u);
    if (bf != T(0) && (prologue ? dzn != 0 : (dzn & lastz) == 0)) {
      const R own = (&ownx[0][0][0])[bix >> 1];
      fxb = fma(bf, lane >= 32 ? IO::hi(own) : IO::lo(own), fxb);
      if constexpr (SH) fxb = fma(bfE, estage[dzn ? b1 : b0][eix], fxb);
    }
  };
  // per lane: all ones, or zero where the neighbouring pair of a slot with
  // sx > 0 (kpos) / sx < 0 (kneg) is a ghost; a slot selects one with its
  // uniform sign and masks the neighbour's dwords (one AND each)
  const uint32_t kpos = lox ? 0u : ~0u, kneg = hix ? 0u : ~0u;
  auto zap = [&](const PairTab &d, R (&v)[4]) {
    const uint32_t k = (d.flags & kPairSxPos) ? kpos : kneg;
    v[1] &= k;
    v[3] &= k;
  };

  // Shifted storage: every slot of a plane interpolates E at the tile's
  // cells and their one-cell halo, of the plane and of the plane above, so
  // the block stages those cells in LDS (kPairSRow) per plane: staged plane
  // j of the range is sp(j) = zb for j = 0, else the plane above zb + j - 1,
  // in ring buffer j % 3; plane zb + k reads buffers k % 3 and (k + 1) % 3.
  // sp(k + 2) is loaded during plane k - 1 and written during plane k,
  // between the barrier after its slot loop (every wave has then finished
  // with the buffer: its last readers are plane k - 1's slot loop and face
  // booking) and the barrier before its collision (plane k + 1 reads it
  // first).  The prologue stages plane zb - 1 in buffer 2 for the carried
  // planes.  Staged column c holds cell x0 - 1 + c wrapped (periodic x) or
  // clamped into the box; a face cell's x-shifted E tap is zeroed like its
  // population's.
  constexpr int KS = SH ? (kPairSPos + 64 * NW - 1) / (64 * NW) : 1;
  uint32_t soff[KS];
  float spend[KS];
  int sb = 0;   // ring buffer of the current plane
  auto stage_ok = [&](int k) { return q * 64 + lane + k * 64 * NW < kPairSPos; };
  if constexpr (SH) {
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      soff[k] = 0u;
      spend[k] = 0.0f;
      if (stage_ok(k)) {
        const int pidx = q * 64 + lane + k * 64 * NW;
        const int r = pidx / kPairSRow;
        int gx = x0 - 1 + (pidx - r * kPairSRow);
        gx = perx ? ((gx % nx) + nx) % nx : min(max(gx, 0), nx - 1);
        soff[k] = (uint32_t)(gx + nx * (y - 1 + r)) * 4u;
      }
    }
  }
  auto stage_load = [&](int64_t plane_cells) {
#pragma unroll
    for (int k = 0; k < KS; ++k)
      if (stage_ok(k))
        spend[k] = ldo<float>(reinterpret_cast<const float *>(ein_bytes) + plane_cells, soff[k]);
  };
  auto stage_write = [&](int b) {
#pragma unroll
    for (int k = 0; k < KS; ++k)
      if (stage_ok(k)) estage[b][1 + q * 64 + lane + k * 64 * NW] = spend[k];
  };
  auto stage_plane = [&](int j) -> int64_t {
    return j == 0 ? (int64_t)zb * pc : plane_above(zb + j - 1);
  };
  // E of both cells of a slot at ring buffer b0 (its new plane is the
  // current one) or b1 (the plane above), from the staged rows y and y - sy:
  // own pair and the one neighbouring cell that the x-shifted taps need
  const int eown = 2 + kPairSRow + 2 * lane;
  auto plane_E = [&](const PairTab &d, int b0, int b1, T &PElo, T &PEhi) {
    const float *eb = &estage[(d.flags & kPairDzn) ? b1 : b0][0];
    const bool pos = (d.flags & kPairSxPos) != 0;
    const int ys = d.row_off > 0 ? kPairSRow : (d.row_off < 0 ? -kPairSRow : 0);
    const int nbo = pos ? -1 : 2;
    const f32x2 a = *reinterpret_cast<const f32x2 *>(eb + eown);
    const f32x2 b = *reinterpret_cast<const f32x2 *>(eb + eown + ys);
    T an = eb[eown + nbo], bn = eb[eown + ys + nbo];
    {
      const uint32_t k = pos ? kpos : kneg;
      an = __uint_as_float(__float_as_uint(an) & k);
      bn = __uint_as_float(__float_as_uint(bn) & k);
    }
    PElo = interp4w(d, a.x, pos ? an : a.y, b.x, pos ? bn : b.y);
    PEhi = interp4w(d, a.y, pos ? a.x : an, b.y, pos ? b.x : bn);
  };
  if constexpr (SH) {
    if (zb < ze) {
      int zl = zb - 1;
      if (perz) zl = wrap(zl, nz);
      stage_load((int64_t)min(max(zl, 0), nz - 1) * pc);
      stage_write(2);
      stage_load(stage_plane(0));
      stage_write(0);
      __syncthreads();
    }
  }

  // prologue: the carried plane value of every slot and both cells (shifted
  // storage: of the population, s_i P + w_i P_E)
  T carry[M][2];
  {
    auto pro = [&]<int J>() {
      const PairTab &d = tb[J];
      carry[J][0] = carry[J][1] = T(0);
      // (sz == 0: the carried plane has weight 0; for sz < 0 it is this
      // block's first plane, whose own values the face cells book)
      if (d.wz_old != T(0) || (d.flags & kPairDzn)) {
        int zl = (d.flags & kPairDzn) ? zb : zb - 1;
        if (perz) zl = wrap(zl, nz);
        R v[4];
        const bool in = (unsigned)zl < (unsigned)nz;
        load4(d, in_bytes + (int64_t)min(max(zl, 0), nz - 1) * pc * SZ, v);
        ownx[q][J][lane] = v[0];
        zap(d, v);
        T a, b;
        interp2(d, v, a, b);
        carry[J][0] = (in ? T(1) : T(0)) * a;
        carry[J][1] = (in ? T(1) : T(0)) * b;
        if constexpr (SH) {
          T ea, eb;
          plane_E(d, 2, 0, ea, eb);
          carry[J][0] = fma(d.w, (in ? T(1) : T(0)) * ea, carry[J][0] * d.scale);
          carry[J][1] = fma(d.w, (in ? T(1) : T(0)) * eb, carry[J][1] * d.scale);
        }
      }
    };
    unroll<0, M>(pro);
  }
  book_face(true, 0, 0, 0);
  if constexpr (SH) {
    if (zb < ze) {
      stage_load(stage_plane(1));
      stage_write(1);
      if (zb + 1 < ze) stage_load(stage_plane(2));
      __syncthreads();
    }
  }

  // the slots of this wave with an inflow ghost plane on an x face that this
  // tile touches (bit J for slot J)
  uint32_t xgmask = 0u;
  if ((p.flags & KF_XGHOSTS) && xface_tile) {
    const bool tlo = x0 == 0, thi = x0 + NC >= nx;
    auto scan = [&]<int J>() {
      const DirTab<T> &d = dtab[q * M + J];
      if (inflow->ghost[q * M + J][0] != nullptr && ((d.s[0] > 0 && tlo) || (d.s[0] < 0 && thi)))
        xgmask |= 1u << J;
    };
    unroll<0, M>(scan);
  }

  __shared__ T red[NW][4][NC];
  __shared__ T coef[SH ? 6 : 5][NC];   // c, alpha, beta (x3); E' (shifted storage)
  R pf[M][4];
  auto issue_first = [&](int zn) {
    const char *const p0 = in_bytes + (int64_t)zn * pc * SZ;
    const char *const p1 = in_bytes + plane_above(zn) * SZ;
    auto one = [&]<int J>() { load4(tb[J], (tb[J].flags & kPairDzn) ? p1 : p0, pf[J]); };
    unroll<0, D>(one);
  };
  if (zb < ze) issue_first(zb);

  // the combine lane's medium, loaded a plane ahead
  T med[3];
  auto load_medium = [&](int64_t cplane, uint32_t om) {
    med[0] = ldo<float>(ka + cplane, om);
    med[1] = ldo<float>(ks + cplane, om);
    med[2] = ldo<float>(eta + cplane, om);
  };
  load_medium((int64_t)zb * pc, ocell * 4u);

  double sE = 0.0, sEs = 0.0;
  const T lam = (T)p.lam;
  const bool lamzero = (p.flags & KF_LAMZERO) != 0;

  for (int z = zb; z < ze; ++z) {
    tb = tab + opaque(q * M);
    const int nv = opaque(p.ndir - q * M);   // this wave's direction slots
    const int64_t cz = (int64_t)z * pc;
    const T kat = med[0], kst = med[1], et = med[2];
    const int64_t cz_next = z + 1 < ze ? cz + pc : cz;
    const uint32_t om = opaque_lane(ocell * 4u);

    // ---- stream: both cells of every slot of this wave
    T Is[M][2];
    T Es[2] = {T(0), T(0)}, F0[2] = {T(0), T(0)}, F1[2] = {T(0), T(0)}, F2[2] = {T(0), T(0)};
    T ref[2] = {T(0), T(0)};
    {
      const char *const p0 = in_bytes + cz * SZ;
      const char *const p1 = in_bytes + plane_above(z) * SZ;
      const int sb1 = sb == 2 ? 0 : sb + 1;   // shifted storage: the plane above
      // plane above the box: vacuum (wave-uniform, so the zeroing is scalar)
      const int gh = __builtin_amdgcn_readfirstlane((!perz && z + 1 >= nz) ? 1 : 0);
      auto slot = [&]<int J>() {
        const PairTab &d = tb[J];
        if constexpr (J + D < M)
          load4(tb[J + D], (tb[J + D].flags & kPairDzn) ? p1 : p0, pf[J + D]);
        ownx[q][J][lane] = pf[J][0];
        zap(d, pf[J]);
        T Pn[2], PE[2];
        interp2(d, pf[J], Pn[0], Pn[1]);
        if constexpr (SH) plane_E(d, sb, sb1, PE[0], PE[1]);
        const T wn = zero_if(d.wz_new, (int)((d.flags >> 1) & 1u) & gh);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          T sv;
          if constexpr (SH) {
            // the population's plane value s_i P + w_i P_E
            const T Ph = fma(d.w, PE[h], Pn[h] * d.scale);
            sv = fma(d.wz_old, carry[J][h], wn * Ph);
            carry[J][h] = Ph;
          } else {
            sv = fma(d.wz_old, carry[J][h], wn * Pn[h]);
            if constexpr (sizeof(S) == 2) sv *= d.scale;
            carry[J][h] = Pn[h];
          }
          Is[J][h] = sv;
          // moments as residuals against the wave's first slot (see accumulate)
          Es[h] += sv;
          if constexpr (J == 0) ref[h] = sv * d.invw;
          const T r = fma(-d.w, ref[h], sv);
          F0[h] = fma(d.n0, r, F0[h]);
          F1[h] = fma(d.n1, r, F1[h]);
          F2[h] = fma(d.n2, r, F2[h]);
        }
      };
      unroll<0, M>(slot);
    }
    if (xgmask != 0u) {
      // Inflow ghosts on the x faces enter after the vacuum sums, slot by
      // slot, for the face cells of the directions with a ghost plane there
      // (as on the other paths, so that all give the same bits).
      auto body = [&]<int J>() {
        if ((xgmask >> J) & 1u) {
          const DirTab<T> &d = dtab[q * M + J];
          const bool pos = d.s[0] > 0;
          if ((pos ? kpos : kneg) == 0u) {
            const T dI = x_ghost_correction<T>(d, inflow->ghost[q * M + J][0], y, z, p.ny, nz,
                                               p.periodic[1], perz);
            fin += (double)dI;
            auto add = [&](int h) {
              Is[J][h] += dI;
              Es[h] += dI;
              F0[h] = fma(d.n[0], dI, F0[h]);
              F1[h] = fma(d.n[1], dI, F1[h]);
              F2[h] = fma(d.n[2], dI, F2[h]);
            };
            if (pos)
              add(0);
            else
              add(1);
          }
        }
      };
      unroll<0, M>(body);
    }

    // ---- the waves' partial sums of the 128 cells
    *reinterpret_cast<f32x2 *>(&red[q][0][2 * lane]) = f32x2{Es[0], Es[1]};
    *reinterpret_cast<f32x2 *>(&red[q][1][2 * lane]) = f32x2{F0[0], F0[1]};
    *reinterpret_cast<f32x2 *>(&red[q][2][2 * lane]) = f32x2{F1[0], F1[1]};
    *reinterpret_cast<f32x2 *>(&red[q][3][2 * lane]) = f32x2{F2[0], F2[1]};
    __syncthreads();

    // ---- combine: item r of this lane is moment j of cell cc (j uniform per wave)
#pragma unroll
    for (int r = 0; r < RI; ++r) {
      const int j = r * (NW / 2) + (q >> 1);
      T v[NW];
#pragma unroll
      for (int w = 0; w < NW; ++w) v[w] = red[w][j][cc];
      const T Sm = tree_sum<T, NW>(v);
      if (j == 0) {
        const CoefE<T> ce = coef_E<T>(p.mode, p.lambda_iters, dt, Sm, kat, kst, et);
        coef[0][cc] = ce.c;
        coef[1][cc] = ce.alpha;
        if constexpr (SH) coef[5][cc] = ce.En;
        if (valid_c) {
          // the new E, part of a shifted state
          if constexpr (SH)
            *reinterpret_cast<float *>(eout_bytes + (cz + ocell) * 4) = ce.En;
          if (p.flags & KF_WRITE_EF) Eout[cz + ocell] = ce.En;
          if (diag) {
            sE += (double)ce.En;
            sEs += (double)Sm;
          }
        }
      } else {
        T Fn, be;
        coef_F<T>(p.mode, p.lambda_iters, dt, lam, Sm, kat, kst, Fn, be);
        coef[1 + j][cc] = be;
        if (valid_c && (p.flags & KF_WRITE_EF)) Fout[(int64_t)(j - 1) * p.ncell + cz + ocell] = Fn;
      }
    }
    // the next plane's medium and first loads go out before the stores
    load_medium(cz_next, om);
    if (z + 1 < ze) issue_first(z + 1);
    if constexpr (SH) {
      // sp(k + 2) into the buffer that plane k - 1 read last; sp(k + 3) loaded
      if (z + 1 < ze) stage_write(sb == 0 ? 2 : sb - 1);
      if (z + 2 < ze) stage_load(stage_plane(z - zb + 3));
    }
    __syncthreads();

    // ---- collide and store both cells of every slot
    const f32x2 c2 = *reinterpret_cast<const f32x2 *>(&coef[0][2 * lane]);
    const f32x2 a2 = *reinterpret_cast<const f32x2 *>(&coef[1][2 * lane]);
    f32x2 b0 = {T(0), T(0)}, b1 = {T(0), T(0)}, b2 = {T(0), T(0)};
    if (!lamzero) {
      b0 = *reinterpret_cast<const f32x2 *>(&coef[2][2 * lane]);
      b1 = *reinterpret_cast<const f32x2 *>(&coef[3][2 * lane]);
      b2 = *reinterpret_cast<const f32x2 *>(&coef[4][2 * lane]);
    }
    f32x2 en2 = {T(0), T(0)};   // shifted storage: both cells' new E
    if constexpr (SH) en2 = *reinterpret_cast<const f32x2 *>(&coef[5][2 * lane]);
    char *const outz = reinterpret_cast<char *>(Iout) + cz * SZ;
    const uint32_t ost = opaque_lane(o0);
    const PairColl *__restrict__ tbc = ctab + opaque(q * M);
    uint32_t g0 = 0u, g1 = 0u;
    if (sizeof(S) == 2 && stoch) {
      const uint32_t cell0 = (uint32_t)(cz + x + nx * y);
      g0 = cell_hash(cell0 ^ p.seed);
      g1 = cell_hash((cell0 + 1u) ^ p.seed);
    }
    // one copy of the slot loop per (lambda = 0, stochastic rounding) pair,
    // so that no slot branches on them
    auto collide_all = [&]<bool LZ, bool SR>() {
#pragma unroll
      for (int jj = 0; jj < M; ++jj) {
        const PairColl &d = tbc[jj];
        if (jj < nv) {   // a direction (null slots come last)
          T o0v = collide_pair(d, c2.x, a2.x, b0.x, b1.x, b2.x, Is[jj][0], LZ);
          T o1v = collide_pair(d, c2.y, a2.y, b0.y, b1.y, b2.y, Is[jj][1], LZ);
          if constexpr (SH) {
            // stored: the deviation from w_i E'
            o0v = fma(-d.w, en2.x, o0v);
            o1v = fma(-d.w, en2.y, o1v);
          }
          if constexpr (sizeof(S) == 2) {
            o0v *= d.inv_scale;
            o1v *= d.inv_scale;
          }
          IO::st(outz + d.plane_off, ost, o0v, o1v, g0 ^ d.rnd, g1 ^ d.rnd, SR);
        }
      }
    };
    if (valid) {
      if (lamzero) {
        if (stoch)
          collide_all.template operator()<true, true>();
        else
          collide_all.template operator()<true, false>();
      } else {
        if (stoch)
          collide_all.template operator()<false, true>();
        else
          collide_all.template operator()<false, false>();
      }
    }
    // this plane's x-face outflux (own values parked during the slot loop;
    // booked here, where the plane's streamed values are no longer live)
    book_face(false, z + 1 >= ze ? 1 : 0, sb, sb == 2 ? 0 : sb + 1);
    sb = sb == 2 ? 0 : sb + 1;
  }

  if (diag) {
    double v[kStepPartials];
#pragma unroll
    for (int k = 0; k < kStepPartials; ++k) v[k] = 0.0;
    v[0] = sE;
    v[1] = sEs;
    v[2] = lane < 32 ? (double)fxb : 0.0;
    v[3] = lane >= 32 ? (double)fxb : 0.0;
    v[8] = fin;
    block_sums<kStepPartials, NW>(v, partials + (int64_t)blockIdx.x * kStepPartials);
  }
}

// Interior tiles of 128 cells, in the XCD-aware block order of the main kernel.
template <typename S, int NB>
__global__ void __launch_bounds__(64 * waves_for(NB), (pair_waves_per_simd<S, NB>()))
step_kernel_pair(const S *__restrict__ Iin, S *__restrict__ Iout, const float *__restrict__ ka,
                 const float *__restrict__ ks, const float *__restrict__ eta,
                 const PairTab *__restrict__ tab, const PairColl *__restrict__ ctab,
                 const DirTab<float> *__restrict__ dtab, const InflowArgs *__restrict__ inflow,
                 const KParams p, float *__restrict__ Eout, float *__restrict__ Fout,
                 double *__restrict__ partials) {
  const int t = xcd_tile(blockIdx.x, p.ntx * p.main_nty);
  const int tix = t % p.ntx;
  const int r = t / p.ntx;
  const int y = p.main_ty0 + r % p.main_nty;
  const int tzr = p.main_zr0 + r / p.main_nty;
  const int zb = tzr * p.zlen;
  march_pair<S, NB>(Iin, Iout, ka, ks, eta, tab, ctab, dtab, inflow, p, Eout, Fout, partials,
                    128 * tix, y, zb, min(p.nz, zb + p.zlen));
}

}  // namespace lbrt
