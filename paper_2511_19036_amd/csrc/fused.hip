// Fused level-sweep kernels for 3-D Poisson with red-black Gauss-Seidel.
//
// Each workgroup owns an x-y tile (64 x TY nodes: one BFP block of 64 per
// row, or two of 32) and marches along z through a chunk of TZ planes.  The
// smoothing stages (half-sweeps) form a pipeline with a lag of one plane per
// stage.  A red-black half-sweep updates one colour and reads only the
// other, and the z-neighbours of a node have the other colour, so every
// plane is updated in place.  The x-y halo covers the dependence cone of the
// stages (redundant work at the tile edges); the z halo costs a few extra
// planes at both ends of a chunk.  Sections are read and written only as BFP
// codes: the finest-level temporaries (the prolongated coarse correction z,
// the decoded solution, the residual) live in registers and LDS.
//
// The per-node arithmetic is exactly that of the per-operation kernels in
// kernels.hip (same operand order, no contraction), so both paths give
// bit-identical results.
//
// Template parameters: S half-sweeps per smoothing kernel (2 nu), TY rows
// and NT threads per tile, LB = log2 of the BFP block (5 or 6), and HI: a
// section read value by value may have a 12- or 64-bit container, so a code
// may straddle two words (the launchers pick HI from the containers; with
// HI = false the second word is neither loaded nor used).  Container-width
// flags of the float64 helpers (C64, W64, GW64) likewise remove the 64-bit
// paths where the launcher knows the container is at most 32 bits.
#include <cmath>
#include <cstdint>
#include <initializer_list>
#include <map>
#include <mutex>
#include <utility>
#include <type_traits>

#include "device.h"
#include "fused.h"
#include "plane.h"
#include "timing.h"

namespace cmg {

constexpr int kTX = 64;

// Tile coordinates of this workgroup (1-D launch over NX * NY * NZ tiles).
// Workgroups are handed to the eight XCDs, each with its own L2, in
// round-robin order of their ids.  The tiles are renumbered so that every
// XCD owns a band of NY / 8 tile rows and walks it x fastest: the x- and
// y-neighbours of a tile, whose halos overlap it, then run on the same L2
// at about the same time, and the halo rows and the partial cache lines at
// the tile's x-edges are fetched from HBM once instead of once per tile.
__device__ __forceinline__ void tile_of(int NX, int NY, int& bx, int& by, int& bz) {
  const int id = blockIdx.x;
  if (NY % 8 != 0) {
    bx = id % NX;
    by = (id / NX) % NY;
    bz = id / (NX * NY);
    return;
  }
  const int x8 = id & 7, sl = id >> 3, band = NY >> 3;
  bx = sl % NX;
  by = x8 * band + (sl / NX) % band;
  bz = sl / (NX * band);
}

__device__ __forceinline__ int ring(int j, int n) { return (j % n + n) % n; }

// d-linear interpolation at fine node (gx, gy, gz) from a coarse ring in LDS
// holding coarse planes cz -> slot ring(cz, NC), tile origin (CX0, CY0),
// width CW.  Same order and weights as prolong_at.
template <typename T, int NC, int CW, int CPL>
__device__ __forceinline__ T prolong_lds(const T* cring, int CX0, int CY0, int gx, int gy, int gz) {
  const int ti = gx >> 1, tj = gy >> 1, tk = gz >> 1;
  const int pi = gx & 1, pj = gy & 1, pk = gz & 1;
  T s = T(0);
  bool first = true;
  for (int oz = 0; oz <= pk; ++oz) {
    const double wz = pk ? 0.5 : 1.0;
    const T* cp = cring + ring(tk + oz, NC) * CPL;
    for (int oy = 0; oy <= pj; ++oy) {
      const double wy = pj ? 0.5 : 1.0;
      for (int ox = 0; ox <= pi; ++ox) {
        const double wx = pi ? 0.5 : 1.0;
        const T t = static_cast<T>(wz * wy * wx) * cp[(tj + oy - CY0) * CW + (ti + ox - CX0)];
        s = first ? t : s + t;
        first = false;
      }
    }
  }
  return s;
}

// A coarse tile [CX0, CX0 + CW) x [CY0, CY0 + CH) of one plane, fetched into
// registers (values outside the level are 0) and later stored into an LDS
// ring slot, so that the loads overlap the work in between.
template <typename T, int CW, int CH, int NT>
struct CoarseFetch {
  static constexpr int N = (CW * CH + NT - 1) / NT;
  T v[N];
  __device__ __forceinline__ void fetch(const T* __restrict__ src, const Geom& gc, int CX0, int CY0, int cz,
                                        int tid) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int t = tid + k * NT;
      const int cy = t / CW, cx = t - cy * CW;
      const int gx = CX0 + cx, gy = CY0 + cy;
      v[k] = T(0);
      if (t < CW * CH && cz >= 0 && cz < gc.n && gx >= 0 && gx < gc.n && gy >= 0 && gy < gc.n)
        v[k] = src[flat(gc, gx, gy, cz)];
    }
  }
  __device__ __forceinline__ void store(T* slot, int tid) const {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int t = tid + k * NT;
      if (t < CW * CH) slot[t] = v[k];
    }
  }
};

// ======================================================= register columns
// Scheme of the down-smoothing kernel.  A workgroup owns an x-y tile of
// 64 x TY output nodes plus a halo of H nodes and marches along z through a
// chunk of TZ planes.  Each thread owns K pairs of adjacent x-columns of
// the extended tile and keeps, per column, a ring of y and right-hand-side
// values of consecutive planes in registers.  The half-sweeps are pipeline
// stages with a lag of one plane.  Stage s updates colour (s + 1) & 1 of its
// plane (red first), so at any one step all stages update the columns of a
// single class (x + y) & 1: the rings are indexed by that class (the slot)
// rather than by the x offset, and with the step loop unrolled by two the
// slot is a compile-time constant.  z-neighbours come from the column's own
// ring; the four in-plane neighbours come from LDS, where every plane under
// way has one buffer: a stage reads the colour that its predecessor wrote at
// the previous step and writes the other colour, so one barrier per step
// suffices.  Nodes near the tile edge outside the dependence cone of the
// output nodes may take inexact values (their LDS reads wrap into the
// neighbouring row or plane) but no node inside the cone reads them.
// Dirichlet boundary nodes and nodes outside the level stay zero.

// Pair geometry of a register-column tile.
template <int H, int TY, int NT>
struct ColTile {
  static constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H;
  static constexpr int PW = EXW / 2, NPAIR = PW * EXH, K = (NPAIR + NT - 1) / NT;
  // plane, its stride (two spare words), margin: the neighbour reads of a
  // missing pair (whose slot is past NPAIR and which works on the spare
  // words) stay inside the LDS array
  static constexpr int LPL = EXW * EXH, PS = LPL + 2, PAD = EXW + 2;
  static constexpr int NW = NT / 64, RPW = (TY + NW - 1) / NW;          // output rows per wave
};

// Output row t of wave wv when TY rows are shared by NW waves.  Waves are
// spread over the four SIMDs round-robin; with NW = 2 (mod 4) SIMDs 2 and 3
// hold one wave fewer, so the rows beyond the first NW go to waves 2, 3, ...
// first (measured: 7% faster up-sweep with 14 waves; no gain for 7).
template <int NW>
__device__ __forceinline__ int out_row(int wv, int t) {
  constexpr int ROT = NW % 4 == 2 ? 2 : 0;
  return t == 0 ? wv : NW * t + (wv - ROT + NW) % NW;
}

// Per-pair flags.
constexpr unsigned kInnerSlot = 0u;  // bits 0, 1: the node of slot s is inside the level's interior
constexpr unsigned kOutSlot = 2u;    // bits 2, 3: the node of slot s is an output node
constexpr unsigned kSwap = 4u;       // bit 4: column 0 holds slot 1

template <int H, int TY, int NT>
__device__ __forceinline__ void col_setup(int tid, int X0, int Y0, int level, int* pos, uint32_t (*xy)[2],
                                          unsigned* fl, int* oidx) {
  using T = ColTile<H, TY, NT>;
  const int n = 1 << level;
#pragma unroll
  for (int k = 0; k < T::K; ++k) {
    const int q = tid + k * NT;
    const bool valid = q < T::NPAIR;
    const int ly = valid ? q / T::PW : 0, lx0 = valid ? 2 * (q - ly * T::PW) : 0;
    const int gx0 = X0 - H + lx0, gy = Y0 - H + ly;
    pos[k] = valid ? ly * T::EXW + lx0 : T::LPL;  // a missing pair writes the spare words
    oidx[k] = (ly - H) * kTX + (lx0 - H);
    const unsigned sw = static_cast<unsigned>(gx0 + gy) & 1u;
    unsigned f = sw << kSwap;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int gx = gx0 + c, lx = lx0 + c;
      const unsigned slot = sw ^ static_cast<unsigned>(c);
      const bool dom = valid && gx >= 0 && gx < n && gy >= 0 && gy < n;
      const bool inner = valid && gx >= 1 && gx < n && gy >= 1 && gy < n;
      const bool out = valid && lx >= H && lx < H + kTX && ly >= H && ly < H + TY;
      xy[k][c] = dom ? ((static_cast<uint32_t>(gy) << level) | static_cast<uint32_t>(gx)) : 0u;
      f |= (inner ? 1u : 0u) << (kInnerSlot + slot);
      f |= (out ? 1u : 0u) << (kOutSlot + slot);
    }
    fl[k] = f;
  }
}

// Quantise the output rows of plane po (tile values in `ob`) into section S.
// The rows of a wave are quantised in one straight-line block (a wave with
// fewer than RPW rows repeats its first row, unstored), then stored.
template <int LB, int TY, int NT, int CB>
__device__ __forceinline__ void quantise_rows(const float* ob, const PSec& S, int po, int X0, int Y0, int level,
                                              int tid) {
  constexpr int NW = NT / 64, RPW = (TY + NW - 1) / NW;
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const PlanePtr pq = plane_at<CB, LB>(S, po, level);
  int m[RPW], e[RPW];
  float v[RPW];
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int rr0 = out_row<NW>(wv, t);
    const int rr = rr0 < TY ? rr0 : out_row<NW>(wv, 0);
    v[t] = ob[rr * kTX + lane];
  }
  quant_f32_rows<LB, RPW>(v, S.w, lane, m, e);
#pragma unroll
  for (int t = 0; t < RPW; ++t) {
    const int rr = out_row<NW>(wv, t);
    if (rr >= TY) continue;
    store_row(pq.c, (static_cast<uint32_t>(Y0 + rr) << level) | static_cast<uint32_t>(X0), lane, m[t], cbits_of<CB>(S));
  }
  if ((lane & ((1 << LB) - 1)) == 0) {
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int rr = out_row<NW>(wv, t);
      if (rr >= TY) continue;
      const uint32_t xyr = (static_cast<uint32_t>(Y0 + rr) << level) | static_cast<uint32_t>(X0);
      pq.e[(xyr + lane) >> LB] = static_cast<int16_t>(e[t]);
    }
  }
}

// =========================================================== down-smoothing
// y'_l = Q(S^nu1(0; g_l)): S = 2 nu1 half-sweeps from zero.  At step j the
// right-hand side of plane j enters and stage s updates plane j - s; the
// first half-sweep is pointwise (y = c g), hence a halo of S - 1.
template <int S, int TY, int NT, int LB, bool HI, int CB>
// (at most 80 VGPRs: two 11-wave workgroups per CU)
__global__ void __launch_bounds__(NT, 6) k_down_smooth(PSec G, PSec Y, int level, float cp, float ih2, int TZ) {
  constexpr int H = S - 1;
  using T = ColTile<H, TY, NT>;
  constexpr int K = T::K, EXW = T::EXW, PS = T::PS, PAD = T::PAD;
  constexpr int NB = S;  // plane j - s is in flight from step j - s + 1 to j - s + S
  __shared__ float lds[2 * PAD + NB * PS];
  __shared__ float outb[2][TY * kTX];
  const int tid = threadIdx.x;
  int bx, by, bz;
  tile_of((1 << level) / kTX, (1 << level) / TY, bx, by, bz);
  const int X0 = bx * kTX, Y0 = by * TY, Z0 = bz * TZ;
  const int n = 1 << level;

  int pos[K], oidx[K];
  uint32_t xy[K][2];
  unsigned fl[K];
  col_setup<H, TY, NT>(tid, X0, Y0, level, pos, xy, fl, oidx);
  int gwm1 = G.w - 1;  // opaque, so that a code's scaling exponent is one subtraction
  auto launder = [&]() {
    opaque_s(gwm1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      opaque(pos[k]);
      opaque(oidx[k]);
      opaque(fl[k]);
      opaque(xy[k][0]);
      opaque(xy[k][1]);
    }
  };

  float y[K][2][S + 2];  // slot-indexed, planes j-S-1 .. j
  float r[K][2][S + 1];  // slot-indexed, planes j-S .. j
  RawCode gpre[K][2];    // column-indexed codes of the next plane
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int i = 0; i < S + 2; ++i) y[k][c][i] = 0.0f;
#pragma unroll
      for (int i = 0; i < S + 1; ++i) r[k][c][i] = 0.0f;
    }
  // Codes of plane p.  Unconditional: a plane outside the level reads
  // plane 1, and its right-hand side is zeroed where it enters.  The words
  // holding the codes are loaded, not the codes themselves (code_at): with
  // the sign-extending loads this kernel took 80 VGPRs and ran 4% slower.
  auto fetch = [&](int p) {
    const PlanePtr gq = plane_at<CB, LB>(G, min(max(p, 1), n - 1), level);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) gpre[k][c] = raw_at<LB, HI>(gq, xy[k][c], cbits_of<CB>(G));
  };

  auto step = [&](auto jpc, const int j) {
    constexpr int JP = decltype(jpc)::value;
    constexpr int SG = 1 - JP;  // slot updated by every stage at this step
    launder();
    // plane j enters: y = 0, rhs from the prefetched codes
    const bool jin = j >= 1 && j < n;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool sw = (fl[k] >> kSwap) & 1u;
      const float g0 = jin ? raw_f32_m1(gpre[k][0], xy[k][0], cbits_of<CB>(G), gwm1) : 0.0f;
      const float g1 = jin ? raw_f32_m1(gpre[k][1], xy[k][1], cbits_of<CB>(G), gwm1) : 0.0f;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int i = 0; i < S + 1; ++i) y[k][c][i] = y[k][c][i + 1];
        y[k][c][S + 1] = 0.0f;
#pragma unroll
        for (int i = 0; i < S; ++i) r[k][c][i] = r[k][c][i + 1];
      }
      r[k][0][S] = sw ? g1 : g0;
      r[k][1][S] = sw ? g0 : g1;
    }
    fetch(j + 1);
    // The plane completed at the previous step is quantised and stored after
    // the codes of plane j were used and those of plane j + 1 requested: a
    // wait for a load does not then include these stores.
    {
      const int po = j - 1 - S;
      if (po >= Z0 && po < Z0 + TZ) quantise_rows<LB, TY, NT, CB>(outb[1 - JP], Y, po, X0, Y0, level, tid);
    }
    // Stage s on plane j - s.  Stages run on every plane of the march: a
    // plane outside the dependence cone of the chunk's output planes is
    // never read by a plane inside it.  (No neighbour pre-loads here, unlike
    // the up sweep: at 80 VGPRs two workgroups share a CU, and the second
    // hides the LDS latency better than pre-loads at 98 VGPRs and one.)
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int p = j - s;
      const bool act = p >= 1 && p < n;
      const int iy = S + 1 - s;
      float* yb = lds + PAD + ((p + 4 * NB) % NB) * PS;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const unsigned sw = (fl[k] >> kSwap) & 1u;
        const int pa = pos[k] + static_cast<int>(static_cast<unsigned>(SG) ^ sw);
        const float yc = y[k][SG][iy];
        const float rhs = r[k][SG][S - s];
        float v;
        if (s == 1) {
          v = cp * rhs;
        } else {
          float a = 6.0f * yc;
          a = a - yb[pa - 1];
          a = a - yb[pa + 1];
          a = a - yb[pa - EXW];
          a = a - yb[pa + EXW];
          a = a - y[k][SG][iy - 1];
          a = a - y[k][SG][iy + 1];
          const float rr = exact_fma(-a, ih2, rhs);  // rhs - a ih2 (ih2 = 4^l)
          v = yc + cp * rr;
        }
        const float yv = (act && ((fl[k] >> (kInnerSlot + SG)) & 1u)) ? v : yc;
        y[k][SG][iy] = yv;
        if (s < S) yb[pa] = yv;
      }
    }
    {
      const int po = j - S;  // both colours have their last update
      if (po >= Z0 && po < Z0 + TZ) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const unsigned sw = (fl[k] >> kSwap) & 1u;
#pragma unroll
          for (int sg = 0; sg < 2; ++sg)
            if ((fl[k] >> (kOutSlot + sg)) & 1u) outb[JP][oidx[k] + static_cast<int>(sg ^ sw)] = y[k][sg][1];
        }
      }
    }
    __syncthreads();
  };

  const int jbeg = Z0 - S, jend = Z0 + TZ + S + 2;  // an even number of steps
  fetch(jbeg);
#pragma unroll 1
  for (int j = jbeg; j < jend; j += 2) {
    step(std::integral_constant<int, 0>(), j);
    step(std::integral_constant<int, 1>(), j + 1);
  }
}

// ============================================================= up-smoothing
// z = P e_{l-1}; rhs = g - A z; y = S^nu2(y'_pre; rhs); Yp = Q(y);
// u'_l = Q(dec u'_l + dec Yp) (float64); e_l = dec Yp + z when eout != null.
//
// Two stages run ahead of the smoother: at step j the columns interpolate z
// of plane j from a ring of coarse planes in LDS and publish it; the
// right-hand side of plane j - 1 then needs the published in-plane z
// neighbours, and the pre-smoothed y' of plane j - 1 is published as stage
// 0.  Stage s updates plane j - 1 - s.  The right-hand side of a node at
// distance d from the output tile needs z at d + 1, and the first half-sweep
// needs y' at d + 1 for d <= S - 1, so the halo is S.
//
// Interpolation weights are powers of two: 2^-(number of odd coordinates);
// the weighted coarse neighbours are summed in C order (z, y, x).  With
// LANEP (the x parity varies over the lanes) every neighbour is added with
// its weight or a zero weight, which is cheaper than selecting the sums: a
// zero term (of a finite value; a non-finite one ends the solve with an
// error) leaves the sum unchanged, as no sum is ever -0 (the coarse values
// are sums of decoded codes, which are +0 or nonzero).  Otherwise (parities
// fixed per column at compile time) the terms are selected.
template <typename T, int PK, int CW, bool LANEP = false>
__device__ __forceinline__ T prolong_node(const T* c0, const T* c1, int ci, bool px, bool py) {
  const T w = (px ? T(0.5) : T(1)) * (py ? T(0.5) : T(1)) * (PK ? T(0.5) : T(1));
  // every weight is a power of two or zero: each product and sum is one
  // exact_fma after the first product
  if (LANEP) {
    const T wx = px ? w : T(0), wy = py ? w : T(0), wxy = (px && py) ? w : T(0);
    T s = w * c0[ci];
    s = exact_fma(c0[ci + 1], wx, s);
    s = exact_fma(c0[ci + CW], wy, s);
    s = exact_fma(c0[ci + CW + 1], wxy, s);
    if (PK) {
      s = exact_fma(c1[ci], w, s);
      s = exact_fma(c1[ci + 1], wx, s);
      s = exact_fma(c1[ci + CW], wy, s);
      s = exact_fma(c1[ci + CW + 1], wxy, s);
    }
    return s;
  }
  T s = w * c0[ci];
  {
    const T t = exact_fma(c0[ci + 1], w, s);
    s = px ? t : s;
  }
  {
    const T t = exact_fma(c0[ci + CW], w, s);
    s = py ? t : s;
  }
  {
    const T t = exact_fma(c0[ci + CW + 1], w, s);
    s = (px && py) ? t : s;
  }
  if (PK) {
    s = exact_fma(c1[ci], w, s);
    {
      const T t = exact_fma(c1[ci + 1], w, s);
      s = px ? t : s;
    }
    {
      const T t = exact_fma(c1[ci + CW], w, s);
      s = py ? t : s;
    }
    {
      const T t = exact_fma(c1[ci + CW + 1], w, s);
      s = (px && py) ? t : s;
    }
  }
  return s;
}

// The same with the y parity PY a compile-time constant and the x parity
// px varying over the lanes: the absent x neighbours are added with a zero
// weight, the absent y neighbours are left out (the same sums: see above).
template <typename T, int PK, int PY, int CW>
__device__ __forceinline__ T prolong_node_x(const T* c0, const T* c1, int ci, bool px) {
  const T w = (px ? T(0.5) : T(1)) * (PY ? T(0.5) : T(1)) * (PK ? T(0.5) : T(1));
  const T wx = px ? w : T(0);
  T s = w * c0[ci];
  s = exact_fma(c0[ci + 1], wx, s);
  if (PY) {
    s = exact_fma(c0[ci + CW], w, s);
    s = exact_fma(c0[ci + CW + 1], wx, s);
  }
  if (PK) {
    s = exact_fma(c1[ci], w, s);
    s = exact_fma(c1[ci + 1], wx, s);
    if (PY) {
      s = exact_fma(c1[ci + CW], w, s);
      s = exact_fma(c1[ci + CW + 1], wx, s);
    }
  }
  return s;
}

// One step of the decode chain, u_l = dec u'_l + P u_{l-1} (float64), at a
// node of level l, for kernels that rebuild the planes of u_l they need
// instead of reading a stored level array (then u_l is never written to
// HBM).  The planes of u_{l-1} under the kernel's coarse footprint pass
// through a ring of three LDS planes (ChainRing, zeros outside the level);
// chain_value forms a node's value with the operand order of the chain's
// own kernel: the decoded code plus the interpolation, whose terms are
// summed in C order (z, y, x) with a zero weight for an absent neighbour.
struct ChainSrc {
  PSec U;            // u'_l (run-time container)
  const double* uc;  // u_{l-1}, level array
  int level;         // l
};
// The LDS ring of u_{l-1} for a coarse footprint of CW x CH nodes of level l
// at (CX0, CY0) (CX0, CY0 >= -1): its parent footprint is CWP x CHP nodes
// at (CX0 >> 1, CY0 >> 1).  fetch/store move plane K (stored at slot
// (K + 3) % 3, K >= -1) through registers so that the loads of one step are
// consumed at its end.
template <int CW, int CH, int NT>
struct ChainRing {
  static constexpr int CWP = CW / 2 + 2, CHP = CH / 2 + 2, PL = CWP * CHP, PT = (PL + NT - 1) / NT;
  double v[PT];
  bool in[PT];
  __device__ __forceinline__ void fetch(const ChainSrc& c, int CX0, int CY0, int K, int tid) {
    const int lp = c.level - 1, np = 1 << lp;
    const bool kin = K >= 0 && K < np;
    const uint32_t kc = static_cast<uint32_t>(min(max(K, 0), np - 1));
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int t = tid + k * NT;
      const int py = t / CWP, px = t - py * CWP;
      const int gx = (CX0 >> 1) + px, gy = (CY0 >> 1) + py;
      in[k] = kin && t < PL && gx >= 0 && gx < np && gy >= 0 && gy < np;
      const uint32_t i = min(max(gx, 0), np - 1), j = min(max(gy, 0), np - 1);
      // the level array of u_{l-1} holds at most 2^27 values: 32-bit byte offsets
      v[k] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(c.uc) +
                                              8u * ((kc << (2 * lp)) | (j << lp) | i));
    }
  }
  __device__ __forceinline__ void store(double* ring, int K, int tid) const {
    double* dst = ring + ((K + 3) % 3) * PL;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int t = tid + k * NT;
      if (t < PL) dst[t] = in[k] ? v[k] : 0.0;
    }
  }
  // Node (gx, gy, gz) of level l (inside it, and inside the footprint at
  // (CX0, CY0)) with code r; the ring holds its parent planes gz >> 1 and
  // (gz >> 1) + 1.
  __device__ __forceinline__ static double value(const ChainSrc& c, const RawCode& r, int gx, int gy, int gz,
                                                 const double* ring, int CX0, int CY0) {
    const uint32_t xy = (static_cast<uint32_t>(gy) << c.level) | static_cast<uint32_t>(gx);
    const double d = raw_f64<true>(r, xy, c.U.cbits, c.U.w);
    const int K = gz >> 1;
    const double* p0 = ring + (K % 3) * PL;
    const double* p1 = ring + ((K + 1) % 3) * PL;
    const int b = ((gy >> 1) - (CY0 >> 1)) * CWP + ((gx >> 1) - (CX0 >> 1));
    const bool px = gx & 1, py = gy & 1, pz = gz & 1;
    const double w = (px ? 0.5 : 1.0) * (py ? 0.5 : 1.0) * (pz ? 0.5 : 1.0);
    const double wx = px ? w : 0.0, wy = py ? w : 0.0, wxy = (px && py) ? w : 0.0;
    double s = w * p0[b];
    s = exact_fma(p0[b + 1], wx, s);
    s = exact_fma(p0[b + CWP], wy, s);
    s = exact_fma(p0[b + CWP + 1], wxy, s);
    s = exact_fma(p1[b], pz ? w : 0.0, s);
    s = exact_fma(p1[b + 1], pz ? wx : 0.0, s);
    s = exact_fma(p1[b + CWP], pz ? wy : 0.0, s);
    s = exact_fma(p1[b + CWP + 1], pz ? wxy : 0.0, s);
    return d + s;
  }
};
template <int LB>
__device__ __forceinline__ RawCode chain_code(const ChainSrc& c, int gx, int gy, int gz) {
  const uint32_t xy = (static_cast<uint32_t>(gy) << c.level) | static_cast<uint32_t>(gx);
  return raw_at<LB, true>(plane_of(c.U, gz), xy, c.U.cbits);
}
// Quads (2 x 2 nodes at even local coordinates) of an up-sweep tile of
// 64 x TY output nodes with halo H, numbered ring by ring: the output tile
// (ring 0, row by row), then ring r = 1 .. H / 2 (the quads r quads outside
// it: bottom row, top row, left column, right column).  Ring r holds the
// nodes at distance 2 r - 1 and 2 r from the output tile.
template <int H, int TY>
__device__ __forceinline__ void quad_of(int t, int& qx, int& qy) {
  constexpr int W0 = kTX / 2, H0 = TY / 2, C = H / 2;  // output quads per row and column; quads of halo
  if (t < W0 * H0) {
    qx = C + t % W0;
    qy = C + t / W0;
    return;
  }
  int before = W0 * H0;
#pragma unroll
  for (int r = 1; r <= C; ++r) {
    const int w = W0 + 2 * r, h = H0 + 2 * r, lo = C - r;
    const int k = t - before;
    if (k >= 0 && k < 2 * w + 2 * (h - 2)) {
      if (k < w) {
        qx = lo + k;
        qy = lo;
      } else if (k < 2 * w) {
        qx = lo + k - w;
        qy = lo + h - 1;
      } else if (k < 2 * w + h - 2) {
        qx = lo;
        qy = lo + 1 + (k - 2 * w);
      } else {
        qx = lo + w - 1;
        qy = lo + 1 + (k - 2 * w - (h - 2));
      }
    }
    before += 2 * w + 2 * (h - 2);
  }
}

// Quads within `dist` nodes of the output tile (the first ones in the
// numbering of quad_of): rings 0 .. (dist + 1) / 2.
template <int H, int TY>
constexpr int cone_quads(int dist) {
  const int r = (dist + 1) / 2 < H / 2 ? (dist + 1) / 2 : H / 2;
  return (kTX / 2 + 2 * r) * (TY / 2 + 2 * r);
}

template <int S, int TY, int NT, int LB, bool HI, int CB>
__global__ void __launch_bounds__(NT, 2) k_up_smooth(const float* __restrict__ ec, PSec G, PSec Y, PSec Yp, PSec U,
                                                     float* __restrict__ eout, int level, int levelc, float cp,
                                                     float ih2, int TZ, int uz) {
  constexpr int H = S;
  static_assert(H % 2 == 0, "even halo: quads start at even coordinates");
  constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H, QW = EXW / 2, QH = EXH / 2, NQ = QW * QH;
  static_assert(NQ <= NT, "one quad per thread");
  // LDS row stride RS: the halo's column quads sit in consecutive lanes two
  // rows apart, 2 RS words, which spreads them over 16 banks (over 4 with
  // RS = EXW).  Plane of the extended tile and its stride: a missing quad
  // works on the two spare rows after the plane.
  constexpr int RS = EXW + 2;
  constexpr int LPL = RS * EXH, PS = LPL + 2 * RS + 2, PAD = RS + 2;
  constexpr int NW = NT / 64, RPW = (TY + NW - 1) / NW;
  constexpr int NB = S + 1;  // y buffers: plane j - 1 - s in flight from step j - s to j - s + S
  // coarse planes: step j reads planes j >> 1 and (j >> 1) + 1 (an odd
  // plane) or only j >> 1 (an even one, which then stores plane (j >> 1) + 1)
  constexpr int NC = 2, CW = QW + 2, CH = QH + 1, CPL = CW * CH, CPT = (CPL + NT - 1) / NT;
  constexpr int OB = TY * kTX + 2 * kTX;  // output tile plus two spare rows (written by the other quads)
  constexpr int NZ = S + 1;               // z of the output tile: planes j - 2 - S .. j - 2
  __shared__ float cs[NC * CPL + 1];      // plus a spare word (written by threads past the coarse tile)
  __shared__ __align__(8) float lds[2 * PAD + (2 + NB) * PS];  // z of planes j, j - 1; then y buffers
  __shared__ __align__(8) float outb[2][OB];
  __shared__ __align__(8) float zo[NZ * OB];  // plane p at slot p mod NZ (NZ = NB: its y buffer index)
  const int tid = threadIdx.x;
  int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int lane = tid & 63;
  int bx, by, bz;
  tile_of((1 << level) / kTX, (1 << level) / TY, bx, by, bz);
  int X0 = bx * kTX, Y0 = by * TY;
  const int Z0 = bz * TZ;
  const int n = 1 << level, nc = 1 << levelc;
  const int CX0 = (X0 - H) >> 1, CY0 = (Y0 - H) >> 1;

  // The quad of this thread: nodes (gx0 + dx, gy0 + dy), dx, dy in {0, 1},
  // node d = dx + 2 dy.  gx0 and gy0 are even, so a node's x and y parities
  // are dx and dy, and its class (x + y) & 1 is dx ^ dy: all compile-time.
  // Threads take the quads ring by ring: first the output tile, then the
  // rings of the halo, so that the later stages (whose dependence cone
  // narrows by one node per stage) skip whole waves.
  const bool valid = tid < NQ;
  int qx = 0, qy = 0;
  if (valid) quad_of<H, TY>(tid, qx, qy);
  const int gx0 = X0 - H + 2 * qx, gy0 = Y0 - H + 2 * qy;
  const bool dom = valid && gx0 >= 0 && gx0 < n && gy0 >= 0 && gy0 < n;  // the quad lies in the level
  int pos = valid ? 2 * qy * RS + 2 * qx : LPL;  // LDS offset of node 0
  int ci = qy * CW + qx;                          // coarse node (gx0 / 2, gy0 / 2) in the coarse ring
  // bits 0-3: node d is an interior node of the level; bit 4: output quad
  unsigned fq = 0u;
  if (dom) {
    fq |= (gx0 >= 1 && gy0 >= 1 ? 1u : 0u) | (gy0 >= 1 ? 2u : 0u) | (gx0 >= 1 ? 4u : 0u) | 8u;
  }
  if (valid && 2 * qx >= H && 2 * qx < H + kTX && 2 * qy >= H && 2 * qy < H + TY) fq |= 16u;
  uint32_t xy0 = dom ? ((static_cast<uint32_t>(gy0) << level) | static_cast<uint32_t>(gx0)) : 0u;
  int oidx = (fq >> 4) & 1u ? (2 * qy - H) * kTX + (2 * qx - H) : TY * kTX;
  int gwm1 = G.w - 1, ywm1 = Y.w - 1;  // opaque: a code's scaling exponent is one subtraction
  auto launder = [&]() {
    opaque(lane);
    opaque_s(gwm1);
    opaque_s(ywm1);
    opaque_s(wv);
    opaque_s(X0);
    opaque_s(Y0);
    opaque_s(level);
    opaque_sec<CB>(G);
    opaque_sec<CB>(Y);
    opaque_sec<CB>(Yp);
    opaque_sec<CB>(U);
    opaque(pos);
    opaque(ci);
    opaque(fq);
    opaque(xy0);
    opaque(oidx);
  };

  float z[4][3];      // planes j-2 .. j
  float r[4][S + 1];  // planes j-1-S .. j-1
  float y[4][S + 2];  // planes j-2-S .. j-1
  RawCode gpre[2], ypre[2], upre[RPW];
  float cpf[CPT];
  bool cin[CPT];
#pragma unroll
  for (int d = 0; d < 4; ++d) {
#pragma unroll
    for (int i = 0; i < 3; ++i) z[d][i] = 0.0f;
#pragma unroll
    for (int i = 0; i < S + 1; ++i) r[d][i] = 0.0f;
#pragma unroll
    for (int i = 0; i < S + 2; ++i) y[d][i] = 0.0f;
  }
  auto cfetch = [&](int cz) {  // coarse tile of plane cz into registers (0 outside the level)
    const bool zin = cz >= 0 && cz < nc;
    const float* src = ec + (static_cast<uint64_t>(zin ? cz : 0) << (2 * levelc));
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      const int cy = t / CW, cx = t - cy * CW;
      const int gx = CX0 + cx, gy = CY0 + cy;
      const bool in = zin && t < CPL && gx >= 0 && gx < nc && gy >= 0 && gy < nc;
      // every lane loads (a node of the level); the value is selected
      const float v = src[(static_cast<uint32_t>(min(max(gy, 0), nc - 1)) << levelc) |
                          static_cast<uint32_t>(min(max(gx, 0), nc - 1))];
      cpf[k] = v;
      cin[k] = in;  // applied where the value is stored: a select here would wait for the load
    }
  };
  auto cstore = [&](int cz) {
    float* dst = cs + (cz & (NC - 1)) * CPL;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      (t < CPL ? dst[t] : cs[NC * CPL]) = cin[k] ? cpf[k] : 0;
    }
  };
  // Codes of the quad's two rows on plane p (G and Y have containers of at
  // most 32 bits: widths of at most 24 with the float32 V-cycle).
  // Unconditional: a plane outside the level reads plane 1, and the
  // right-hand side part zeroes its values.
  auto fetch_gy = [&](int p) {
    const int pc = min(max(p, 1), n - 1);
    const PlanePtr gq = plane_at<CB, LB>(G, pc, level), yq = plane_at<CB, LB>(Y, pc, level);
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const uint32_t xr = xy0 + (static_cast<uint32_t>(dy) << level);
      gpre[dy] = pair_code_at<CB, LB>(gq, xr, cbits_of<CB>(G));
      ypre[dy] = pair_code_at<CB, LB>(yq, xr, cbits_of<CB>(Y));
    }
  };
  // Rows of a wave: out_row(wv, t) for t < RPW; a wave with fewer than RPW
  // rows repeats its first row in the missing slots (computed, not stored),
  // so that the quantisation of all its rows is one straight-line block.
  auto row_of = [&](int t) {
    const int rr = out_row<NW>(wv, t);
    return rr < TY ? rr : out_row<NW>(wv, 0);
  };
  // Codes of the output rows of plane po.  Unconditional (a plane outside
  // the chunk reads a chunk plane, unused): the loads are only waited for at
  // the next step, after the stores issued before them.
  auto fetch_u = [&](int po) {
    const PlanePtr uq = plane_at<CB, LB>(U, min(max(po, Z0), Z0 + TZ - 1), level);
#pragma unroll
    for (int t = 0; t < RPW; ++t)
      upre[t] = code_at<CB, LB, HI>(uq, ((static_cast<uint32_t>(Y0 + row_of(t)) << level) | X0) + lane, cbits_of<CB>(U));
  };
  // Output plane po: quantise y' (Yp), correct u' (float64), e = dec Yp + z.
  // The arithmetic of all rows of the wave is one straight-line block
  // (finish_compute); the stores follow in finish_store, issued after the
  // loads of the step so that no wait for those loads includes them.
  struct Fin {
    int my[RPW], ey[RPW], eu[RPW];
    int64_t mu[RPW];
    float ev[RPW];
  };
  auto finish_compute = [&](int po, const float* ob, const float* zb, Fin& F) {
    if (po < Z0 || po >= Z0 + TZ) return;
    // the rows are quantised together (their DPP reductions interleave)
    float yv[RPW];
#pragma unroll
    for (int t = 0; t < RPW; ++t) yv[t] = ob[row_of(t) * kTX + lane];
    quant_f32_rows<LB, RPW>(yv, Yp.w, lane, F.my, F.ey);
    double vu[RPW];
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const uint32_t xyl = ((static_cast<uint32_t>(Y0 + row_of(t)) << level) | static_cast<uint32_t>(X0)) + lane;
      const double dy = ldexp(static_cast<double>(F.my[t]), F.ey[t] - (Yp.w - 1));  // codes 0 in a zero block
      // uz: u' holds zeros that were never written (its first correction
      // on this FMG level): the codes read are not used
      vu[t] = (uz ? 0.0 : code_f64<CB, may64<CB, HI>()>(upre[t], xyl, cbits_of<CB>(U), U.w)) + dy;
      F.ev[t] = static_cast<float>(dy);
    }
    quant_f64_rows<LB, may64<CB, HI>(), RPW>(vu, U.wq, lane, F.mu, F.eu);
    if (eout != nullptr) {  // z of the plane, kept since its own step
#pragma unroll
      for (int t = 0; t < RPW; ++t) F.ev[t] = F.ev[t] + zb[row_of(t) * kTX + lane];
    }
  };
  // Yp is stored only when the caller keeps it (no buffers otherwise).
  const bool keep = Yp.codes != nullptr;
  auto finish_store = [&](int po, const Fin& F) {
    if (po < Z0 || po >= Z0 + TZ) return;
    const PlanePtr yq = plane_at<CB, LB>(Yp, po, level), uq = plane_at<CB, LB>(U, po, level);
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int rr = out_row<NW>(wv, t);
      if (rr >= TY) continue;
      const uint32_t xyr = (static_cast<uint32_t>(Y0 + rr) << level) | static_cast<uint32_t>(X0);
      if (keep) store_row(yq.c, xyr, lane, F.my[t], cbits_of<CB>(Yp));
      store_row(uq.c, xyr, lane, F.mu[t], cbits_of<CB>(U));
      if (eout != nullptr)  // the plane's base, then a 32-bit offset in it
        *reinterpret_cast<float*>(reinterpret_cast<char*>(eout + (static_cast<uint64_t>(po) << (2 * level))) +
                                  4u * (xyr + static_cast<uint32_t>(lane))) = F.ev[t];
    }
    // every lane of a block stores the block's exponent (the same value to
    // the same address): no branch on the lane
#pragma unroll
    for (int t = 0; t < RPW; ++t) {
      const int rr = out_row<NW>(wv, t);
      if (rr >= TY) continue;
      const uint32_t xyl = ((static_cast<uint32_t>(Y0 + rr) << level) | static_cast<uint32_t>(X0)) + lane;
      if (keep) yq.e[xyl >> LB] = static_cast<int16_t>(F.ey[t]);
      uq.e[xyl >> LB] = static_cast<int16_t>(F.eu[t]);
    }
  };

  // bj: the y buffer index of plane j - 1, (j - 1) mod NB, carried by the loop
  auto step = [&](auto jpc, const int j, const int bj) {
    constexpr int JP = decltype(jpc)::value;  // every stage updates the nodes of class JP at this step
    launder();
    // y buffer of plane j - 1 - s (0 <= s <= S < NB)
    auto ybuf = [&](int s) { return lds + PAD + (2 + bj - s + (bj < s ? NB : 0)) * PS; };
    // z ring (NZ = NB): plane j - 2 - S = j - 1 - NB at slot bj, plane j - 2 at slot bj - 1
    float* const zfin = zo + bj * OB;
    float* const znew = zo + (bj == 0 ? NB - 1 : bj - 1) * OB;
    {
      Fin F;
      finish_compute(j - 2 - S, outb[1 - JP], zfin, F);
      fetch_u(j - 1 - S);
      if (JP == 1) cfetch((j + 3) >> 1);  // stored at the next step: z(j + 2) needs coarse plane (j + 3) / 2
      finish_store(j - 2 - S, F);
    }
    {  // z of plane j
      const float* c0 = cs + ((j >> 1) & (NC - 1)) * CPL;
      const float* c1 = cs + (((j >> 1) + 1) & (NC - 1)) * CPL;
      float* zb = lds + PAD + JP * PS;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        z[d][0] = z[d][1];
        z[d][1] = z[d][2];
        z[d][2] = prolong_node<float, JP, CW>(c0, c1, ci, (d & 1) != 0, (d & 2) != 0);
      }
      *reinterpret_cast<float2*>(zb + pos) = make_float2(z[0][2], z[1][2]);
      *reinterpret_cast<float2*>(zb + pos + RS) = make_float2(z[2][2], z[3][2]);
      // z of plane j - 2 on the output tile (the other quads write the spare
      // rows), read when the plane is finished
      *reinterpret_cast<float2*>(&znew[oidx]) = make_float2(z[0][0], z[1][0]);
      *reinterpret_cast<float2*>(&znew[oidx + kTX]) = make_float2(z[2][0], z[3][0]);
    }
    {  // plane j - 1: rhs = g - A z, and y' as stage 0
      const int p = j - 1;
      const bool pin = p >= 1 && p < n;
      const float* zs = lds + PAD + (1 - JP) * PS;
      float* yb = ybuf(0);
      // in-plane neighbours outside the quad: x - 1 / x + 1 of the left /
      // right column, y - 1 / y + 1 of the lower / upper row
      const float zxm0 = zs[pos - 1], zxm2 = zs[pos + RS - 1];
      const float zxp1 = zs[pos + 2], zxp3 = zs[pos + RS + 2];
      const float zym0 = zs[pos - RS], zym1 = zs[pos - RS + 1];
      const float zyp2 = zs[pos + 2 * RS], zyp3 = zs[pos + 2 * RS + 1];
      float rv[4], yv[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int dx = d & 1, dy = d >> 1;
        const float xm = dx ? z[d ^ 1][1] : (dy ? zxm2 : zxm0);
        const float xp = dx ? (dy ? zxp3 : zxp1) : z[d ^ 1][1];
        const float ym = dy ? z[d ^ 2][1] : (dx ? zym1 : zym0);
        const float yp = dy ? (dx ? zyp3 : zyp2) : z[d ^ 2][1];
        float a = 6.0f * z[d][1];
        a = a - xm;
        a = a - xp;
        a = a - ym;
        a = a - yp;
        a = a - z[d][0];
        a = a - z[d][2];
        const bool kp = pin && ((fq >> d) & 1u);
        const uint32_t xr = xy0 + (static_cast<uint32_t>(dy) << level);
        const float gv = exact_fma(-a, ih2, pair_code_f32<CB>(gpre[dy], xr, dx, cbits_of<CB>(G), gwm1));
        const float y0 = pair_code_f32<CB>(ypre[dy], xr, dx, cbits_of<CB>(Y), ywm1);
        rv[d] = kp ? gv : 0.0f;
        yv[d] = kp ? y0 : 0.0f;
      }
      *reinterpret_cast<float2*>(yb + pos) = make_float2(yv[0], yv[1]);
      *reinterpret_cast<float2*>(yb + pos + RS) = make_float2(yv[2], yv[3]);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int i = 0; i < S; ++i) r[d][i] = r[d][i + 1];
#pragma unroll
        for (int i = 0; i < S + 1; ++i) y[d][i] = y[d][i + 1];
        r[d][S] = rv[d];
        y[d][S + 1] = yv[d];
      }
      fetch_gy(j);
    }
    // Post-smoothing: stage s on plane j - 1 - s updates the two nodes of
    // class JP of the quad (d = 0, 3 or d = 1, 2); of the four in-plane
    // neighbours of a node two are in the quad (registers) and two in the
    // neighbouring quads (LDS, written by stage s - 1 at the previous step).
    // As in the down sweep, stages run on every plane of the march.  Stage s
    // matters only within S - s nodes of the output tile: waves whose quads
    // all lie farther out skip it (their values there are never read by a
    // node that matters).
    constexpr int DA = JP == 0 ? 0 : 1, DB = JP == 0 ? 3 : 2;  // the two nodes of class JP
    float nb[2][4];  // outer neighbours of node DA (x, y) and DB (x, y), stage s + 1 loaded ahead
    auto load_stage = [&](int s, float (&v)[4]) {
      const float* yb = ybuf(s);
      if (JP == 0) {  // node 0: x - 1, y - 1; node 3: x + 1, y + 1
        v[0] = yb[pos - 1];
        v[1] = yb[pos - RS];
        v[2] = yb[pos + RS + 2];
        v[3] = yb[pos + 2 * RS + 1];
      } else {  // node 1: x + 1, y - 1; node 2: x - 1, y + 1
        v[0] = yb[pos + 2];
        v[1] = yb[pos - RS + 1];
        v[2] = yb[pos + RS - 1];
        v[3] = yb[pos + 2 * RS];
      }
    };
    auto stage_on = [&](int s) { return 64 * wv < cone_quads<H, TY>(S - s); };
    if (stage_on(1)) load_stage(1, nb[0]);
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      if (!stage_on(s)) continue;
      if (s < S && stage_on(s + 1)) load_stage(s + 1, nb[s & 1]);
      const int p = j - 1 - s;
      if (p < 1 || p >= n) continue;  // a plane outside the level keeps its zeros
      const int iy = S + 1 - s;
      float* yb = ybuf(s);
      const float* o = nb[(s - 1) & 1];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int d = h == 0 ? DA : DB;
        const int dx = d & 1, dy = d >> 1;
        const float ox = o[2 * h], oy = o[2 * h + 1];
        const float xm = dx ? y[d ^ 1][iy] : ox;
        const float xp = dx ? ox : y[d ^ 1][iy];
        const float ym = dy ? y[d ^ 2][iy] : oy;
        const float yp = dy ? oy : y[d ^ 2][iy];
        const float yc = y[d][iy];
        float a = 6.0f * yc;
        a = a - xm;
        a = a - xp;
        a = a - ym;
        a = a - yp;
        a = a - y[d][iy - 1];
        a = a - y[d][iy + 1];
        const float rr = exact_fma(-a, ih2, r[d][S - s]);
        const float v = yc + cp * rr;
        const float yv = ((fq >> d) & 1u) ? v : yc;
        y[d][iy] = yv;
        if (s < S) yb[pos + dy * RS + dx] = yv;
      }
    }
    // plane j - 1 - S is complete: into the output buffer (read at the next
    // step when the plane lies in the chunk; quads outside the output tile
    // write the spare rows)
    *reinterpret_cast<float2*>(&outb[JP][oidx]) = make_float2(y[0][1], y[1][1]);
    *reinterpret_cast<float2*>(&outb[JP][oidx + kTX]) = make_float2(y[2][1], y[3][1]);
    if (JP == 0) cstore((j + 2) >> 1);
    __syncthreads();
  };

  const int jbeg = Z0 - S, jend = Z0 + TZ + S + 2;  // an even number of steps
  cfetch(jbeg >> 1);
  cstore(jbeg >> 1);
  cfetch((jbeg + 2) >> 1);
  fetch_gy(jbeg - 1);
  __syncthreads();
  int bj = (jbeg - 1 + 4 * NB) % NB;
#pragma unroll 1
  for (int j = jbeg; j < jend; j += 2) {
    step(std::integral_constant<int, 0>(), j, bj);
    bj = bj == NB - 1 ? 0 : bj + 1;
    step(std::integral_constant<int, 1>(), j + 1, bj);
    bj = bj == NB - 1 ? 0 : bj + 1;
  }
}

// ======================================================== residual-restrict
// g_{l-1} = Q(R(g_l - A y'_l)) on a coarse tile of 64 x CTY nodes, marching
// along the fine planes.  Three stages with a lag of one plane each, one
// barrier per step:
//   A: the threads decode y' of fine plane s for their own columns of the
//      fine tile (plus a halo of two) and publish it (ring of three planes);
//   B: t = g - A y' on plane s - 1 for the own columns inside the t region
//      (z-neighbours from the column's registers), published (two planes);
//   C: each coarse node adds the nine weighted t values of plane s - 2 to
//      its running full-weighting sum (the 27 terms in C order: z, y, x);
//      on an odd fine plane 2K + 1 the sum of coarse plane K is complete and
//      the sum of plane K + 1 starts with the same nine products.
// The t planes are stored split by x parity so that the stride-two reads of
// the coarse nodes are consecutive.
template <int CTY, int NT, int LB, bool HI, int CB>
__global__ void __launch_bounds__(NT) k_resid_restrict(PSec G, PSec Y, PSec Gc, int level, float ih2, int TZc) {
  constexpr int YW = 2 * kTX + 4, YH = 2 * CTY + 3;  // y' region, origin (2 CX0 - 2, 2 CY0 - 2)
  constexpr int NCOL = YW * YH, YPS = NCOL + 1, K = (NCOL + NT - 1) / NT;
  constexpr int TW = 2 * kTX + 2, TH = 2 * CTY + 1, TPL = TW * TH;  // t region, origin (2 CX0 - 1, 2 CY0 - 1)
  constexpr int TPS = TPL + 1, YPAD = YW + 1;  // a spare word per plane; margins for the edge columns' reads
  constexpr int NW = NT / 64, CRW = CTY / NW;
  static_assert(CTY % NW == 0, "whole coarse rows per wave");
  __shared__ float yl[2 * YPAD + 3 * YPS];
  __shared__ float tl[2 * TPS];
  const int tid = threadIdx.x;
  int lane = tid & 63;
  int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int bx, by, bz;
  tile_of((1 << (level - 1)) / kTX, (1 << (level - 1)) / CTY, bx, by, bz);
  int CX0 = bx * kTX, CY0 = by * CTY;
  const int CZ0 = bz * TZc;
  const int n = 1 << level, levelc = level - 1;

  int pos[K], tpos[K];
  uint32_t xy[K];
  unsigned fl[K];  // bit 0: node in the level; bit 1: t column; bit 2: interior node
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = tid + k * NT;
    const bool valid = q < NCOL;
    const int ly = valid ? q / YW : 0, lx = valid ? q - ly * YW : 0;
    const int gx = 2 * CX0 - 2 + lx, gy = 2 * CY0 - 2 + ly;
    const bool dom = valid && gx >= 0 && gx < n && gy >= 0 && gy < n;
    const bool inner = valid && gx >= 1 && gx < n && gy >= 1 && gy < n;
    const bool tcol = valid && lx >= 1 && lx <= TW && ly >= 1 && ly <= TH;
    pos[k] = valid ? q : NCOL;
    const int tx = lx - 1, ty = ly - 1;
    tpos[k] = tcol ? ty * TW + (tx & 1) * (TW / 2) + (tx >> 1) : TPL;
    xy[k] = dom ? ((static_cast<uint32_t>(gy) << level) | static_cast<uint32_t>(gx)) : 0u;
    fl[k] = (dom ? 1u : 0u) | (tcol ? 2u : 0u) | (inner ? 4u : 0u);
  }
  // Every column slot computes: a slot past NCOL works on the spare words
  // (plane offset 0 for its loads), so that no load sits under a branch.
  float yr[K][3];  // y' of planes s-2 .. s
  RawCode ypre[K], gpre[K];
  float sc[CRW];   // running coarse sums
#pragma unroll
  for (int k = 0; k < K; ++k) yr[k][0] = yr[k][1] = yr[k][2] = 0.0f;
#pragma unroll
  for (int r = 0; r < CRW; ++r) sc[r] = 0.0f;
  // Codes of plane p (a plane outside the level reads a level plane; the
  // stages zero the values of planes outside it).
  auto fetch_y = [&](int p) {
    const PlanePtr yq = plane_at<CB, LB>(Y, min(max(p, 0), n - 1), level);
#pragma unroll
    for (int k = 0; k < K; ++k) ypre[k] = code_at<CB, LB, HI>(yq, xy[k], cbits_of<CB>(Y));
  };
  auto fetch_g = [&](int p) {
    const PlanePtr gq = plane_at<CB, LB>(G, min(max(p, 1), n - 1), level);
#pragma unroll
    for (int k = 0; k < K; ++k) gpre[k] = code_at<CB, LB, HI>(gq, xy[k], cbits_of<CB>(G));
  };

  int ywm1 = Y.w - 1, gwm1 = G.w - 1;
  auto step = [&](auto spc, const int s) {
    constexpr int SP = decltype(spc)::value;  // parity of s and of the plane s - 2 of stage C
    opaque(lane);
    opaque_s(ywm1);
    opaque_s(gwm1);
    opaque_s(wv);
    opaque_s(CX0);
    opaque_s(CY0);
    opaque_sec<CB>(G);
    opaque_sec<CB>(Y);
    opaque_sec<0>(Gc);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      opaque(pos[k]);
      opaque(tpos[k]);
      opaque(xy[k]);
    }
    {  // A: y' of plane s
      const bool pin = s >= 0 && s < n;
      float* yb = yl + YPAD + ((s + 3) % 3) * YPS;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        yr[k][0] = yr[k][1];
        yr[k][1] = yr[k][2];
        const float v = code_f32<CB>(ypre[k], xy[k], cbits_of<CB>(Y), ywm1);
        yr[k][2] = (pin && (fl[k] & 1u)) ? v : 0.0f;
        yb[pos[k]] = yr[k][2];
      }
    }
    {  // B: t on plane s - 1
      const int p = s - 1;
      const bool pin = p >= 1 && p < n;
      const float* ya = yl + YPAD + ((p + 3) % 3) * YPS;
      float* tb = tl + ((p + 2) & 1) * TPS;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int c = pos[k];
        float a = 6.0f * yr[k][1];
        a = a - ya[c - 1];
        a = a - ya[c + 1];
        a = a - ya[c - YW];
        a = a - ya[c + YW];
        a = a - yr[k][0];
        a = a - yr[k][2];
        const float v = exact_fma(-a, ih2, code_f32<CB>(gpre[k], xy[k], cbits_of<CB>(G), gwm1));
        tb[tpos[k]] = (pin && (fl[k] & 4u)) ? v : 0.0f;
      }
    }
    fetch_y(s + 1);
    fetch_g(s);
    {  // C: plane q = s - 2 into the coarse sums
      const int q = s - 2;
      const float* ta = tl + ((q + 2) & 1) * TPS;
      const float wz = SP ? 0.25f : 0.5f;
#pragma unroll
      for (int r = 0; r < CRW; ++r) {
        const int jr = wv + NW * r;  // coarse row within the tile
        float prod[9];
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
          const float* trow = ta + (2 * jr + oy + 1) * TW;
          const float wy = oy == 0 ? 0.5f : 0.25f;
          const float t0 = trow[lane];                // x = 2I - 1
          const float t1 = trow[TW / 2 + lane];       // x = 2I
          const float t2 = trow[lane + 1];            // x = 2I + 1
          prod[3 * (oy + 1) + 0] = (wz * wy * 0.25f) * t0;
          prod[3 * (oy + 1) + 1] = (wz * wy * 0.5f) * t1;
          prod[3 * (oy + 1) + 2] = (wz * wy * 0.25f) * t2;
        }
        if (SP == 0) {  // oz = 0 of coarse plane q / 2
#pragma unroll
          for (int i = 0; i < 9; ++i) sc[r] = sc[r] + prod[i];
        } else {  // oz = +1 of plane (q - 1) / 2, then oz = -1 of plane (q + 1) / 2
          float done = sc[r];
#pragma unroll
          for (int i = 0; i < 9; ++i) done = done + prod[i];
          float next = prod[0];
#pragma unroll
          for (int i = 1; i < 9; ++i) next = next + prod[i];
          sc[r] = next;
          const int Kc = (q - 1) >> 1;
          if (Kc >= CZ0 && Kc < CZ0 + TZc) {
            const int J = CY0 + jr, I = CX0 + lane;
            const float v = (I >= 1 && J >= 1 && Kc >= 1) ? done : 0.0f;
            const PlanePtr cq = plane_of(Gc, Kc);
            const uint32_t xyr = (static_cast<uint32_t>(J) << levelc) | static_cast<uint32_t>(CX0);
            int e;
            const int m = quant_f32<LB>(v, Gc.w, lane, &e);
            store_row(cq.c, xyr, lane, m, Gc.cbits);
            if ((lane & ((1 << LB) - 1)) == 0) cq.e[(xyr + lane) >> LB] = static_cast<int16_t>(e);
          }
        }
      }
    }
    __syncthreads();
  };

  const int sbeg = 2 * CZ0 - 2, send = 2 * (CZ0 + TZc) + 2;  // an even number of steps, sbeg even
  fetch_y(sbeg);
  fetch_g(sbeg - 1);
#pragma unroll 1
  for (int s0 = sbeg; s0 < send; s0 += 2) {
    step(std::integral_constant<int, 0>(), s0);
    step(std::integral_constant<int, 1>(), s0 + 1);
  }
}

// ============================================================= IR residual
// g_Lp = Q(f - A(dec u'_Lp + P u_{Lp-1})) in float64 (Alg. 2 on the finest
// level of the current FMG level); f is the caller's full node array of the
// finest level L, sampled with stride 2^(L - Lp).
//
// Each thread owns RPT output columns (x = X0 + lane, rows wv + NW t) and
// keeps u of planes j-2 .. j of them in registers; the threads tid < NHALO
// also decode one node of the one-node x-y halo.  Every plane of u goes
// through a ring of three LDS planes, so that a single barrier per step
// separates the writes of plane j from the reads of plane j - 2.
template <int TY, int NT, int XW, int LB, bool HI, bool GW64, int CB, bool SKIP>
__global__ void __launch_bounds__(NT) k_ir_residual(PSec U, const double* __restrict__ uc,
                                                    const double* __restrict__ f, int Lfull, int level, int levelc,
                                                    double ih2, PSec Gout, int TZ, int* nonfinite, double* sumsq,
                                                    ChainSrc ch, int uz) {
  // XW blocks of 64 side by side: wave wv owns block wv % XW of rows
  // wv / XW + NWR t
  constexpr int TXW = kTX * XW, NW = NT / 64, NWR = NW / XW, RPT = TY / NWR;
  static_assert(NW % XW == 0 && TY % NWR == 0, "whole rows per wave");
  constexpr int EXW = TXW + 2, LPL = EXW * (TY + 2);
  constexpr int NHALO = 2 * EXW + 2 * TY;
  static_assert(NHALO <= NT, "one halo node per thread");
  constexpr int NC = 4, CW = TXW / 2 + 3, CH = TY / 2 + 3, CPL = CW * CH, CPT = (CPL + NT - 1) / NT;
  using Ring = ChainRing<CW, CH, NT>;
  __shared__ double us[3 * LPL];
  __shared__ double cs[NC * CPL];
  __shared__ double ps[SKIP ? 3 * Ring::PL : 1];  // SKIP: planes of u_{Lp-2}
  const int tid = threadIdx.x;
  int lane = tid & 63;
  int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int xl = lane + kTX * (tid / 64 % XW);                          // tile-local x of the lane
  int wr = __builtin_amdgcn_readfirstlane(tid / 64 / XW);          // first row of the wave
  int xb = __builtin_amdgcn_readfirstlane(kTX * (tid / 64 % XW));  // tile-local x of its block
  int bx, by, bz;
  tile_of((1 << level) / TXW, (1 << level) / TY, bx, by, bz);
  int X0 = bx * TXW, Y0 = by * TY;
  const int Z0 = bz * TZ;
  const int n = 1 << level, nc = 1 << levelc;
  const int CX0 = (X0 >> 1) - 1, CY0 = (Y0 >> 1) - 1;
  const int64_t N = (static_cast<int64_t>(1) << Lfull) + 1;
  const int fst = 1 << (Lfull - level);

  // halo node of this thread (tile-local hx in -1..TXW, hy in -1..TY)
  int hx = 0, hy = 0;
  if (tid < EXW) {
    hy = -1;
    hx = tid - 1;
  } else if (tid < 2 * EXW) {
    hy = TY;
    hx = tid - EXW - 1;
  } else if (tid < 2 * EXW + TY) {
    hx = -1;
    hy = tid - 2 * EXW;
  } else {
    hx = TXW;
    hy = tid - 2 * EXW - TY;
  }
  const bool has_h = tid < NHALO;
  int gxh = X0 + hx, gyh = Y0 + hy;
  const bool hdom = has_h && gxh >= 0 && gxh < n && gyh >= 0 && gyh < n;
  uint32_t xyh = hdom ? ((static_cast<uint32_t>(gyh) << level) | static_cast<uint32_t>(gxh)) : 0u;
  int hpos = has_h ? (hy + 1) * EXW + hx + 1 : 0;
  int hci = ((gyh >> 1) - CY0) * CW + ((gxh >> 1) - CX0);

  double u[RPT][3];
  RawCode upre[RPT], hpre;
  double fpre[RPT];
  double cpf[CPT];
  bool cin[CPT];
  RawCode ccode[SKIP ? CPT : 1];  // SKIP: u_{Lp-1} is rebuilt from u'_{Lp-1} and u_{Lp-2}
  Ring ring;
#pragma unroll
  for (int t = 0; t < RPT; ++t) u[t][0] = u[t][1] = u[t][2] = 0.0;
  auto xy_own = [&](int t) {
    return (static_cast<uint32_t>(Y0 + wr + NWR * t) << level) | static_cast<uint32_t>(X0 + xl);
  };
  // the node of coarse slot t, clamped into the level
  auto cnode = [&](int t, int& gx, int& gy) {
    const int cy = t / CW, cx = t - cy * CW;
    gx = CX0 + cx;
    gy = CY0 + cy;
  };
  auto cfetch = [&](int cz) {
    const bool zin = cz >= 0 && cz < nc;
    const double* src = uc + (static_cast<uint64_t>(zin ? cz : 0) << (2 * levelc));
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      int gx, gy;
      cnode(t, gx, gy);
      const bool in = zin && t < CPL && gx >= 0 && gx < nc && gy >= 0 && gy < nc;
      // every lane loads (a node of the level); the value is selected
      const int gxc = min(max(gx, 0), nc - 1), gyc = min(max(gy, 0), nc - 1);
      if (SKIP) {
        ccode[k] = chain_code<LB>(ch, gxc, gyc, zin ? cz : 0);
      } else {
        const double v = src[(static_cast<uint32_t>(gyc) << levelc) | static_cast<uint32_t>(gxc)];
        cpf[k] = v;
      }
      cin[k] = in;  // applied where the value is stored: a select here would wait for the load
    }
  };
  auto cstore = [&](int cz) {
    double* dst = cs + (cz & (NC - 1)) * CPL;
    const bool zin = cz >= 0 && cz < nc;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      if (t < CPL) {
        double v;
        if (SKIP) {
          int gx, gy;
          cnode(t, gx, gy);
          v = Ring::value(ch, ccode[k], min(max(gx, 0), nc - 1), min(max(gy, 0), nc - 1), zin ? cz : 0, ps, CX0,
                          CY0);
        } else {
          v = cpf[k];
        }
        dst[t] = cin[k] ? v : 0;
      }
    }
  };
  // The loads below are unconditional (a plane outside the level reads a
  // level plane, a halo node outside it reads node 0, f on the boundary is
  // read and replaced): a load under a branch makes the compiler wait for
  // it, and for every memory operation issued before it, where the
  // branches join.  The consumers zero what lies outside.
  auto fetch_u = [&](int p) {
    const PlanePtr uq = plane_at<CB, LB>(U, min(max(p, 0), n - 1), level);
#pragma unroll
    for (int t = 0; t < RPT; ++t) upre[t] = code_at<CB, LB, HI>(uq, xy_own(t), cbits_of<CB>(U));
    hpre = code_at<CB, LB, HI>(uq, xyh, cbits_of<CB>(U));
  };
  auto fetch_f = [&](int p) {  // f at the own columns of plane p
    const double* fp = f + static_cast<uint64_t>(min(max(p, 0), n - 1)) * fst * N * N;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int gx = X0 + xl, gy = Y0 + wr + NWR * t;
      const double v =
          fp[static_cast<uint32_t>(gy * fst) * static_cast<uint32_t>(N) + static_cast<uint32_t>(gx * fst)];
      fpre[t] = v;  // boundary values are read but not used (the residual zeroes them)
    }
  };

  double acc = 0.0;  // sum of squares of this thread's residuals (monitor)
  auto step = [&](auto jpc, const int j) {
    constexpr int JP = decltype(jpc)::value;
    opaque(lane);
    opaque(xl);
    opaque_s(wr);
    opaque_s(xb);
    opaque(xyh);
    opaque(hpos);
    opaque(hci);
    opaque(gxh);
    opaque(gyh);
    opaque_s(wv);
    opaque_s(X0);
    opaque_s(Y0);
    opaque_sec<CB>(U);
    opaque_sec<CB>(Gout);
    if (JP == 0) {
      cfetch((j + 2) >> 1);  // u(j + 1) needs coarse plane (j + 2) / 2
      if (SKIP) ring.fetch(ch, CX0, CY0, (((j + 2) >> 1) >> 1) + 2, tid);  // its parent planes run 2 ahead
    }
    {  // u of plane j
      const bool pin = j >= 0 && j < n;
      const double* c0 = cs + ((j >> 1) & (NC - 1)) * CPL;
      const double* c1 = cs + (((j >> 1) + 1) & (NC - 1)) * CPL;
      double* ub = us + ((j + 3) % 3) * LPL;
      // the rows of a wave are NWR (even) apart: their y parity is the
      // wave's, a compile-time constant in each branch
      auto own = [&](auto pyc) {
        constexpr int PY = decltype(pyc)::value;
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const int rr = wr + NWR * t;
          u[t][0] = u[t][1];
          u[t][1] = u[t][2];
          const int ci = ((rr >> 1) + 1) * CW + (xl >> 1) + 1;
          // uz: u' holds zeros that were never written (the first IR
          // iteration of an FMG level): the codes read are not used
          const double v = (uz ? 0.0 : code_f64<CB, may64<CB, HI>()>(upre[t], xy_own(t), cbits_of<CB>(U), U.w)) +
                           prolong_node_x<double, JP, PY, CW>(c0, c1, ci, lane & 1);
          u[t][2] = pin ? v : 0.0;
          ub[(rr + 1) * EXW + xl + 1] = u[t][2];
        }
      };
      static_assert(NWR % 2 == 0, "rows of one parity per wave");
      if (wr & 1) own(std::integral_constant<int, 1>());
      else own(std::integral_constant<int, 0>());
      if (has_h) {
        const double v =
            (uz ? 0.0 : code_f64<CB, may64<CB, HI>()>(hpre, xyh, cbits_of<CB>(U), U.w)) +
            prolong_node<double, JP, CW, true>(c0, c1, hci, gxh & 1, gyh & 1);
        ub[hpos] = (pin && hdom) ? v : 0.0;
      }
    }
    fetch_u(j + 1);
    if (JP == 0) {
      cstore((j + 2) >> 1);
      if (SKIP) ring.store(ps, (((j + 2) >> 1) >> 1) + 2, tid);
    }
    __syncthreads();
    const int p = j - 1;
    if (p >= Z0 && p < Z0 + TZ) {  // residual on plane p
      const double* ua = us + ((p + 3) % 3) * LPL;
      const PlanePtr gq = plane_at<CB, LB>(Gout, p, level);
      // all rows are quantised in one straight-line block, then stored
      double tv[RPT];
      int64_t m[RPT];
      int e[RPT];
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int rr = wr + NWR * t;
        const int c = (rr + 1) * EXW + xl + 1;
        double a = 6.0 * u[t][1];
        a = a - ua[c - 1];
        a = a - ua[c + 1];
        a = a - ua[c - EXW];
        a = a - ua[c + EXW];
        a = a - u[t][0];
        a = a - u[t][2];
        const bool inside = p >= 1 && X0 + xl >= 1 && Y0 + rr >= 1;
        tv[t] = inside ? exact_fma(-a, ih2, fpre[t]) : 0.0;
      }
      quant_f64_rows<LB, GW64, RPT>(tv, Gout.w, lane, m, e);
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const uint32_t xyr = (static_cast<uint32_t>(Y0 + wr + NWR * t) << level) | static_cast<uint32_t>(X0 + xb);
        store_row(gq.c, xyr, lane, m[t], cbits_of<CB>(Gout));
      }
      if ((lane & ((1 << LB) - 1)) == 0) {
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const uint32_t xyr = (static_cast<uint32_t>(Y0 + wr + NWR * t) << level) | static_cast<uint32_t>(X0 + xb);
          gq.e[(xyr + lane) >> LB] = static_cast<int16_t>(e[t]);
        }
      }
      if (nonfinite != nullptr) {
        bool bad = false;
#pragma unroll
        for (int t = 0; t < RPT; ++t) bad = bad || !isfinite(tv[t]);
        if (bad) atomicOr(nonfinite, 1);
      }
#pragma unroll
      for (int t = 0; t < RPT; ++t) acc = acc + tv[t] * tv[t];
    }
    fetch_f(j);
  };

  const int jbeg = Z0 - 1, jend = Z0 + TZ + 1;  // an even number of steps, jbeg odd
  if (SKIP) {  // the parent planes of the first two coarse planes and of the first step's
#pragma unroll 1
    for (int K = (jbeg >> 1) >> 1; K <= ((jbeg >> 1) >> 1) + 2; ++K) {
      ring.fetch(ch, CX0, CY0, K, tid);
      ring.store(ps, K, tid);
    }
    __syncthreads();
  }
  cfetch(jbeg >> 1);
  cstore(jbeg >> 1);
  cfetch((jbeg >> 1) + 1);
  cstore((jbeg >> 1) + 1);
  fetch_u(jbeg);
  fetch_f(jbeg - 1);  // unused: gives the first step the same loads in flight as every later one
  __syncthreads();
#pragma unroll 1
  for (int j = jbeg; j < jend; j += 2) {
    step(std::integral_constant<int, 1>(), j);
    step(std::integral_constant<int, 0>(), j + 1);
  }
  if (sumsq != nullptr) monitor_add(sumsq, acc);  // the residual monitor's slots
}

// ============================================================ final decode
// u (full node grid of level l) = dec u'_l + P u_{l-1}; far boundary 0.
// A z-march like the residual: each thread owns one column of a 64 x TY
// tile, coarse planes come through a ring in LDS, and every plane is
// written as whole rows.  Tiles at the far x / y edges also write the
// boundary column / row at node 2^l; the last chunk writes plane 2^l.
// PAD: write the padded level layout (2^l per axis) instead, as one step of
// the decode chain u_l = dec u'_l + P u_{l-1}.  SKIP: u_{l-1} is rebuilt
// from u'_{l-1} and u_{l-2} (ch) where it is needed; uc is not read.
template <int TY, int LB, bool PAD, bool HI, int CB, bool SKIP>
__global__ void __launch_bounds__(64 * TY) k_decode_full(PSec U, const double* __restrict__ uc, int level,
                                                         int levelc, int TZ, double* __restrict__ full,
                                                         ChainSrc ch) {
  constexpr int NT = 64 * TY;
  constexpr int NC = 4, CW = kTX / 2 + 2, CH = TY / 2 + 2, CPL = CW * CH, CPT = (CPL + NT - 1) / NT;
  using Ring = ChainRing<CW, CH, NT>;
  __shared__ double cs[NC * CPL];
  __shared__ double ps[SKIP ? 3 * Ring::PL : 1];  // SKIP: planes of u_{l-2}
  const int tid = threadIdx.x;
  int lane = tid & 63;
  int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int bx, by, bz;
  tile_of((1 << level) / kTX, (1 << level) / TY, bx, by, bz);
  int X0 = bx * kTX, Y0 = by * TY;
  const int Z0 = bz * TZ;
  const int n = 1 << level, nc = 1 << levelc;
  const uint64_t N = static_cast<uint64_t>(n) + (PAD ? 0 : 1);
  const int CX0 = X0 >> 1, CY0 = Y0 >> 1;
  double cpf[CPT];
  bool cin[CPT];
  RawCode ccode[SKIP ? CPT : 1];
  Ring ring;
  RawCode upre;
  auto cfetch = [&](int cz) {
    const bool zin = cz >= 0 && cz < nc;
    const double* src = uc + (static_cast<uint64_t>(zin ? cz : 0) << (2 * levelc));
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      const int cy = t / CW, cx = t - cy * CW;
      const int gx = CX0 + cx, gy = CY0 + cy;
      const bool in = zin && t < CPL && gx < nc && gy < nc;
      // every lane loads (a node of the level); the value is selected
      if (SKIP) {
        ccode[k] = chain_code<LB>(ch, min(gx, nc - 1), min(gy, nc - 1), zin ? cz : 0);
      } else {
        const double v =
            src[(static_cast<uint32_t>(min(gy, nc - 1)) << levelc) | static_cast<uint32_t>(min(gx, nc - 1))];
        cpf[k] = v;
      }
      cin[k] = in;  // applied where the value is stored: a select here would wait for the load
    }
  };
  auto cstore = [&](int cz) {
    double* dst = cs + (cz & (NC - 1)) * CPL;
    const bool zin = cz >= 0 && cz < nc;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int t = tid + k * NT;
      if (t < CPL) {
        double v;
        if (SKIP) {
          const int cy = t / CW, cx = t - cy * CW;
          v = Ring::value(ch, ccode[k], min(CX0 + cx, nc - 1), min(CY0 + cy, nc - 1), zin ? cz : 0, ps, CX0, CY0);
        } else {
          v = cpf[k];
        }
        dst[t] = cin[k] ? v : 0;
      }
    }
  };
  auto xy_own = [&]() { return (static_cast<uint32_t>(Y0 + wv) << level) | static_cast<uint32_t>(X0 + lane); };
  auto fetch_u = [&](int k) {  // unconditional: past the last plane it reads that plane again, unused
    upre = code_at<CB, LB, HI>(plane_at<CB, LB>(U, min(k, n - 1), level), xy_own(), cbits_of<CB>(U));
  };
  auto step = [&](auto kpc, const int k) {
    constexpr int KP = decltype(kpc)::value;
    opaque(lane);
    opaque_s(wv);
    opaque_s(X0);
    opaque_s(Y0);
    opaque_sec<CB>(U);
    if (KP == 0) {
      cfetch((k >> 1) + 1);  // plane k + 1 needs coarse plane k / 2 + 1
      if (SKIP) ring.fetch(ch, CX0, CY0, (((k >> 1) + 1) >> 1) + 2, tid);  // its parent planes run 2 ahead
    }
    const RawCode r = upre;
    fetch_u(k + 1);
    const double* c0 = cs + ((k >> 1) & (NC - 1)) * CPL;
    const double* c1 = cs + (((k >> 1) + 1) & (NC - 1)) * CPL;
    const int ci = (wv >> 1) * CW + (lane >> 1);
    const double v =
        code_f64<CB, may64<CB, HI>()>(r, xy_own(), cbits_of<CB>(U), U.w) + prolong_node<double, KP, CW, true>(c0, c1, ci, lane & 1, wv & 1);
    double* row = full + (static_cast<uint64_t>(k) * N + static_cast<uint64_t>(Y0 + wv)) * N;
    row[X0 + lane] = v;  // (the faces at 2^l of a full array are written by k_far_faces)
    if (KP == 0) {
      cstore((k >> 1) + 1);
      if (SKIP) ring.store(ps, (((k >> 1) + 1) >> 1) + 2, tid);
    }
    __syncthreads();
  };
  if (SKIP) {  // the parent planes of the first coarse plane and of the first step's
#pragma unroll 1
    for (int K = (Z0 >> 1) >> 1; K <= ((Z0 >> 1) >> 1) + 2; ++K) {
      ring.fetch(ch, CX0, CY0, K, tid);
      ring.store(ps, K, tid);
    }
    __syncthreads();
  }
  cfetch(Z0 >> 1);
  cstore(Z0 >> 1);
  fetch_u(Z0);
  __syncthreads();
#pragma unroll 1
  for (int k = Z0; k < Z0 + TZ; k += 2) {
    step(std::integral_constant<int, 0>(), k);
    step(std::integral_constant<int, 1>(), k + 1);
  }
}

// The Dirichlet faces x = 2^l, y = 2^l and z = 2^l of a full node array
// (N = 2^l + 1 per axis) are zero; the z-march above writes the rest, with
// no conditional store in its loop.
__global__ void k_far_faces(double* __restrict__ full, int n) {
  const uint64_t N = static_cast<uint64_t>(n) + 1, face = N * N;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < 3 * face;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t f = i / face, r = i - f * face, a = r / N, b = r - a * N;
    const uint64_t off = f == 0 ? (a * N + b) * N + n : f == 1 ? (a * N + n) * N + b : (n * N + a) * N + b;
    full[off] = 0.0;
  }
}

// =============================================================== launchers
// Workgroups of `kernel` (launched with nthreads threads) that the device
// holds at once: resident workgroups per CU times the CUs.  Cached per
// device and kernel.
static int resident_slots(const void* kernel, int nthreads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, kernel);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nthreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  return cache[key] = per_cu * cus;
}

// Planes per workgroup (chunk) of a z-march over n planes and tiles_xy
// tiles.  A workgroup's run time is about proportional to the steps it
// takes, step_mul * tz + halo_steps (its chunk plus the z-halo), and a
// launch takes one such time per round of workgroups over the resident
// slots.  The chunk, a power of two from 2 to n, minimises rounds x steps;
// ties go to the longer chunk (less redundant halo work).  Small levels get
// short chunks (their launches are latency bound), large ones few rounds.
// On levels of 512 planes or more the launch keeps at least min_rounds
// rounds where it can: workgroups that share a CU then run out of phase
// (measured at 1024^3: the float64 residual and the restriction are 5-8%
// faster with four rounds than with one; the smoothing sweeps are fastest
// with two).
static int chunk_planes(const void* kernel, int nthreads, int n, int tiles_xy, int step_mul, int halo_steps,
                        int min_rounds) {
  const int64_t slots = resident_slots(kernel, nthreads);
  int best = n;
  int64_t best_cost = INT64_MAX;
  for (int pass = 0; pass < 2 && best_cost == INT64_MAX; ++pass) {
    for (int tz = n; tz >= 2; tz >>= 1) {
      const int64_t wgs = static_cast<int64_t>(tiles_xy) * (n / tz), rounds = (wgs + slots - 1) / slots;
      if (pass == 0 && n >= 512 && rounds < min_rounds) continue;
      const int64_t cost = rounds * (static_cast<int64_t>(step_mul) * tz + halo_steps);
      if (cost < best_cost) {
        best_cost = cost;
        best = tz;
      }
    }
  }
  return best;
}

static double sec_b(const SecRef& s) {
  const double nb = static_cast<double>((s.n + s.B - 1) / s.B);
  return nb * s.B * s.cbits / 8.0 + 2.0 * nb;
}

#define CMG_FLAUNCH(name, nbytes, kernel, grid, block, stream, ...)                                 \
  do {                                                                                             \
    if (g_timing != nullptr) g_timing->begin((name), static_cast<double>(nbytes), stream, g.level); \
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                      \
    if (g_timing != nullptr) g_timing->end(stream);                                       \
  } while (0)

constexpr int kDownTY = 32, kUpTY = 32, kResTY = 32, kRRCTY = 8, kDownNT = 704, kUpNT = 768, kResNT = 512,
              kRRNT = 512, kDecTY = 8;

// Container shared by the sections a kernel reads value by value, when the
// kernels have a compile-time variant for it (8, 12, 16 or 32 bits), else 0.
static int common_cb(std::initializer_list<const SecRef*> ss) {
  const int cb = (*ss.begin())->cbits;
  for (const SecRef* s : ss)
    if (s->cbits != cb) return 0;
  return (cb == 8 || cb == 12 || cb == 16 || cb == 32) ? cb : 0;
}

// Launch L(..., HI, CB) with CB = cb for the compile-time containers (the
// 12-bit one with straddling codes), else the run-time variant.
#define CMG_BY_CB(L, hi, cb, ...)                      \
  do {                                                 \
    if (hi && (cb) == 12) L(__VA_ARGS__, true, 12);    \
    else if (hi) L(__VA_ARGS__, true, 0);              \
    else if ((cb) == 8) L(__VA_ARGS__, false, 8);      \
    else if ((cb) == 16) L(__VA_ARGS__, false, 16);    \
    else if ((cb) == 32) L(__VA_ARGS__, false, 32);    \
    else L(__VA_ARGS__, false, 0);                     \
  } while (0)

static PSec psec(const SecRef& s, const Geom& g) {
  const uint64_t pv = static_cast<uint64_t>(1) << (2 * g.level);  // values per plane
  PSec p;
  p.codes = static_cast<char*>(s.codes);
  p.exps = s.exps;
  p.plane_bytes = static_cast<uint32_t>(pv * s.cbits / 8);
  p.plane_blks = static_cast<uint32_t>(pv / s.B);
  p.cbits = s.cbits;
  p.w = s.w;
  p.wq = corr_width(s);
  return p;
}

// The kernels contract the products with h^-2 into exact_fma: h^-2 must be
// a power of two (4^l on the unit cube), else the per-operation kernels run.
static bool pow2_scale(double v) {
  int e;
  return v > 0.0 && std::frexp(v, &e) == 0.5;
}

bool fused_down_smooth(const SecRef& G, const SecRef& Y, const Geom& g, int nu, float cp, float ih2,
                       hipStream_t st) {
  if (g.dim != 3 || g.n < kTX || (nu != 1 && nu != 2) || (G.B != 32 && G.B != 64) || Y.B != G.B || !pow2_scale(ih2))
    return false;
  const int tiles = (g.n / kTX) * (g.n / kDownTY);
  const dim3 block(kDownNT);
  const double bytes = sec_b(G) + sec_b(Y);
  const PSec pg = psec(G, g), py = psec(Y, g);
  const bool hi = G.cbits == 12;
  const int cb = common_cb({&G, &Y});
#define CMG_DOWN(S_, LB_, HI_, CB_)                                                                             \
  do {                                                                                                        \
    const int tz = chunk_planes(reinterpret_cast<const void*>(&k_down_smooth<S_, kDownTY, kDownNT, LB_, HI_, CB_>), \
                                kDownNT, g.n, tiles, 1, 2 * (S_) + 2, 2);                                        \
    CMG_FLAUNCH("k_down_smooth<" #S_ ">", bytes, (k_down_smooth<S_, kDownTY, kDownNT, LB_, HI_, CB_>),           \
                dim3(tiles * (g.n / tz)), block, st, pg, py, g.level, cp, ih2, tz);                           \
  } while (0)
  if (nu == 2) {
    if (G.B == 64) CMG_BY_CB(CMG_DOWN, hi, cb, 4, 6);
    else CMG_BY_CB(CMG_DOWN, hi, cb, 4, 5);
  } else {
    if (G.B == 64) CMG_BY_CB(CMG_DOWN, hi, cb, 2, 6);
    else CMG_BY_CB(CMG_DOWN, hi, cb, 2, 5);
  }
#undef CMG_DOWN
  return true;
}

bool fused_up_smooth(const float* ec, const SecRef& G, const SecRef& Y, const SecRef& Yp, const SecRef& U,
                     float* eout, const Geom& g, const Geom& gc, int nu, float cp, float ih2, hipStream_t st,
                     bool u_zero) {
  if (g.dim != 3 || g.n < kTX || (nu != 1 && nu != 2) || (G.B != 32 && G.B != 64) || Y.B != G.B || Yp.B != G.B ||
      U.B != G.B || !pow2_scale(ih2))
    return false;
  const int tiles = (g.n / kTX) * (g.n / kUpTY);
  const dim3 block(kUpNT);
  const double bytes = sec_b(G) + sec_b(Y) + (Yp.codes != nullptr ? sec_b(Yp) : 0.0) + 2.0 * sec_b(U) +
                       4.0 * gc.size + (eout ? 4.0 * g.size : 0.0);
  const PSec pg = psec(G, g), py = psec(Y, g), pp = psec(Yp, g), pu = psec(U, g);
  const bool hi = U.cbits == 12 || U.cbits == 64;  // the codes of u' may straddle two words
  const int cb = common_cb({&G, &Y, &Yp, &U});
#define CMG_UP(S_, LB_, HI_, CB_)                                                                                \
  do {                                                                                                           \
    const int tz = chunk_planes(reinterpret_cast<const void*>(&k_up_smooth<S_, kUpTY, kUpNT, LB_, HI_, CB_>), kUpNT, \
                                g.n, tiles, 1, 2 * (S_) + 2, 2);                                                 \
    CMG_FLAUNCH("k_up_smooth<" #S_ ">", bytes, (k_up_smooth<S_, kUpTY, kUpNT, LB_, HI_, CB_>),                     \
                dim3(tiles * (g.n / tz)), block, st, ec, pg, py, pp, pu, eout, g.level, gc.level, cp, ih2, tz,   \
                u_zero ? 1 : 0);                                                                                 \
  } while (0)
  if (nu == 2) {
    if (G.B == 64) CMG_BY_CB(CMG_UP, hi, cb, 4, 6);
    else CMG_BY_CB(CMG_UP, hi, cb, 4, 5);
  } else {
    if (G.B == 64) CMG_BY_CB(CMG_UP, hi, cb, 2, 6);
    else CMG_BY_CB(CMG_UP, hi, cb, 2, 5);
  }
#undef CMG_UP
  return true;
}

bool fused_resid_restrict(const SecRef& G, const SecRef& Y, const SecRef& Gc, const Geom& g, const Geom& gc,
                          float ih2, hipStream_t st) {
  if (g.dim != 3 || gc.n < kTX || (G.B != 32 && G.B != 64) || Y.B != G.B || Gc.B != G.B || !pow2_scale(ih2)) return false;
  const int tiles = (gc.n / kTX) * (gc.n / kRRCTY);
  const dim3 block(kRRNT);
  const double bytes = sec_b(G) + sec_b(Y) + sec_b(Gc);
  const PSec pg = psec(G, g), py = psec(Y, g), pc = psec(Gc, gc);
  const bool hi = G.cbits == 12 || Y.cbits == 12;
  const int cb = common_cb({&G, &Y});
#define CMG_RR(LB_, HI_, CB_)                                                                                   \
  do {                                                                                                          \
    const int tz = chunk_planes(reinterpret_cast<const void*>(&k_resid_restrict<kRRCTY, kRRNT, LB_, HI_, CB_>), \
                                kRRNT, gc.n, tiles, 2, 4, 4);                                                      \
    CMG_FLAUNCH("k_resid_restrict", bytes, (k_resid_restrict<kRRCTY, kRRNT, LB_, HI_, CB_>),                      \
                dim3(tiles * (gc.n / tz)), block, st, pg, py, pc, g.level, ih2, tz);                            \
  } while (0)
  if (G.B == 64) CMG_BY_CB(CMG_RR, hi, cb, 6);
  else CMG_BY_CB(CMG_RR, hi, cb, 5);
#undef CMG_RR
  return true;
}

bool fused_ir_residual(const SecRef& U, const double* uc, const double* f, int Lfull, const Geom& g, const Geom& gc,
                       double ih2, const SecRef& Gout, int* nonfinite, double* sumsq, hipStream_t st,
                       const SecRef* Uc, const double* ucc, bool u_zero) {
  if (g.dim != 3 || g.n < kTX || (U.B != 32 && U.B != 64) || Gout.B != U.B || !pow2_scale(ih2)) return false;
  const bool skip = Uc != nullptr;
  if (skip && (Uc->B != U.B || gc.level < 4 || ucc == nullptr)) return false;
  // tiles of two blocks side by side from 128 nodes per row: half the
  // partial 128-byte lines at the x-edges of the rows of f and the halos
  const bool wide = g.n >= 2 * kTX;
  const int tiles = (g.n / (wide ? 2 * kTX : kTX)) * (g.n / kResTY);
  const double coarse = skip ? sec_b(*Uc) + 8.0 * (gc.size >> 3) : 8.0 * gc.size;
  const double bytes = sec_b(U) + coarse + 8.0 * g.size + sec_b(Gout);
  const PSec pu = psec(U, g), pg = psec(Gout, g);
  ChainSrc ch{};
  if (skip) ch = ChainSrc{psec(*Uc, gc), ucc, gc.level};
  const bool hi = U.cbits == 12 || U.cbits == 64, g64 = Gout.cbits == 64;
  const int cb = common_cb({&U, &Gout});
#define CMG_IRS(XW_, LB_, HI_, GW_, CB_, SK_)                                                                    \
  do {                                                                                                          \
    constexpr int nt_ = kResNT * (XW_);                                                                         \
    const int tz = chunk_planes(                                                                                \
        reinterpret_cast<const void*>(&k_ir_residual<kResTY, nt_, XW_, LB_, HI_, GW_, CB_, SK_>), nt_, g.n,      \
        tiles, 1, 2, 4);                                                                                        \
    CMG_FLAUNCH("k_ir_residual", bytes, (k_ir_residual<kResTY, nt_, XW_, LB_, HI_, GW_, CB_, SK_>),             \
                dim3(tiles * (g.n / tz)), dim3(nt_), st, pu, uc, f, Lfull, g.level, gc.level, ih2, pg, tz,      \
                nonfinite, sumsq, ch, u_zero ? 1 : 0);                                                          \
  } while (0)
#define CMG_IRX(XW_, LB_, HI_, GW_, CB_)                 \
  do {                                                   \
    if (skip) CMG_IRS(XW_, LB_, HI_, GW_, CB_, true);     \
    else CMG_IRS(XW_, LB_, HI_, GW_, CB_, false);         \
  } while (0)
#define CMG_IR(LB_, HI_, GW_, CB_)                   \
  do {                                               \
    if (wide) CMG_IRX(2, LB_, HI_, GW_, CB_);         \
    else CMG_IRX(1, LB_, HI_, GW_, CB_);              \
  } while (0)
#define CMG_IRG(LB_, HI_, CB_)          \
  do {                                  \
    if (g64) CMG_IR(LB_, HI_, true, 0); \
    else CMG_IR(LB_, HI_, false, CB_);  \
  } while (0)
#define CMG_IR2(LB_) CMG_BY_CB(CMG_IRG, hi, cb, LB_)
  if (U.B == 64) {
    CMG_IR2(6);
  } else {
    CMG_IR2(5);
  }
#undef CMG_IRG
#undef CMG_IR2
#undef CMG_IR
#undef CMG_IRX
#undef CMG_IRS
  return true;
}

bool fused_decode_full(const SecRef& U, const double* uc, const Geom& g, const Geom& gc, double* full,
                       hipStream_t st, const SecRef* Uc, const double* ucc) {
  if (g.dim != 3 || g.n < kTX || (U.B != 32 && U.B != 64)) return false;
  const bool skip = Uc != nullptr;
  if (skip && (Uc->B != U.B || gc.level < 4 || ucc == nullptr)) return false;
  const int64_t N = g.n + 1;
  const double coarse = skip ? sec_b(*Uc) + 8.0 * (gc.size >> 3) : 8.0 * gc.size;
  const double bytes = sec_b(U) + coarse + 8.0 * N * N * N;
  const PSec pu = psec(U, g);
  ChainSrc ch{};
  if (skip) ch = ChainSrc{psec(*Uc, gc), ucc, gc.level};
  const int tiles = (g.n / kTX) * (g.n / kDecTY);
  const dim3 block(64 * kDecTY);
  const bool hi = U.cbits == 12 || U.cbits == 64;
  const int cb = common_cb({&U});
#define CMG_DECS(LB_, HI_, CB_, SK_)                                                                            \
  do {                                                                                                         \
    const int tz = chunk_planes(reinterpret_cast<const void*>(&k_decode_full<kDecTY, LB_, false, HI_, CB_, SK_>), \
                                64 * kDecTY, g.n, tiles, 1, 2, 1);                                                \
    CMG_FLAUNCH("k_decode_full", bytes, (k_decode_full<kDecTY, LB_, false, HI_, CB_, SK_>),                     \
                dim3(tiles * (g.n / tz)), block, st, pu, uc, g.level, gc.level, tz, full, ch);                 \
  } while (0)
#define CMG_DEC(LB_, HI_, CB_)                  \
  do {                                          \
    if (skip) CMG_DECS(LB_, HI_, CB_, true);     \
    else CMG_DECS(LB_, HI_, CB_, false);         \
  } while (0)
  if (U.B == 64) CMG_BY_CB(CMG_DEC, hi, cb, 6);
  else CMG_BY_CB(CMG_DEC, hi, cb, 5);
#undef CMG_DEC
#undef CMG_DECS
  hipLaunchKernelGGL(k_far_faces, dim3(1024), dim3(256), 0, st, full, g.n);
  return true;
}

bool fused_decode_level(const SecRef& U, const double* uc, const Geom& g, const Geom& gc, double* out,
                        hipStream_t st) {
  if (g.dim != 3 || g.n < kTX || (U.B != 32 && U.B != 64)) return false;
  const double bytes = sec_b(U) + 8.0 * gc.size + 8.0 * g.size;
  const PSec pu = psec(U, g);
  const int tiles = (g.n / kTX) * (g.n / kDecTY);
  const dim3 block(64 * kDecTY);
  const bool hi = U.cbits == 12 || U.cbits == 64;
  const int cb = common_cb({&U});
#define CMG_DEC(LB_, HI_, CB_)                                                                                  \
  do {                                                                                                         \
    const int tz = chunk_planes(reinterpret_cast<const void*>(&k_decode_full<kDecTY, LB_, true, HI_, CB_, false>), \
                                64 * kDecTY, g.n, tiles, 1, 2, 1);                                                \
    CMG_FLAUNCH("k_decode_level", bytes, (k_decode_full<kDecTY, LB_, true, HI_, CB_, false>),                     \
                dim3(tiles * (g.n / tz)), block, st, pu, uc, g.level, gc.level, tz, out, ChainSrc{});          \
  } while (0)
  if (U.B == 64) CMG_BY_CB(CMG_DEC, hi, cb, 6);
  else CMG_BY_CB(CMG_DEC, hi, cb, 5);
#undef CMG_DEC
  return true;
}

}  // namespace cmg
