// Fused level-sweep kernels for 3-D Poisson with red-black Gauss-Seidel.
//
// Each workgroup owns an x-y tile (64 x TY nodes: one BFP block of 64 per
// row, or two of 32) and marches along z through a chunk of TZ planes,
// keeping a ring of planes in LDS.  The smoothing stages (half-sweeps) form
// a pipeline with a lag of one plane per stage: at step j the plane j is
// loaded and stage s updates plane j - s.  A red-black half-sweep updates
// one colour and reads only the other, and the z-neighbours of a colour are
// of the other colour, so every plane is updated in place.  The x-y halo
// shrinks by one node per stage (redundant work at the tile edges); the z
// halo costs S extra planes at both ends of a chunk.  Sections are read and
// written only as BFP codes: the finest-level temporaries (the prolongated
// coarse correction z, the decoded solution, the residual) live in LDS.
//
// LDS planes are split by the parity of the tile-local x index (even and
// odd halves), so that lanes updating one colour touch consecutive words.
//
// The per-node arithmetic is exactly that of the per-operation kernels in
// kernels.hip (same operand order, no contraction), so both paths give
// bit-identical results.
#include "device.h"
#include "fused.h"
#include "timing.h"

namespace cmg {

constexpr int kTX = 64;

__device__ __forceinline__ int ring(int j, int n) { return (j % n + n) % n; }

// Tile-local plane addressing with the x-parity split.
template <int EXW, int EXH>
struct Plane {
  static constexpr int W2 = EXW / 2;
  static constexpr int SIZE = EXW * EXH;
  __device__ static __forceinline__ int at(int lx, int ly) { return ((lx & 1) * EXH + ly) * W2 + (lx >> 1); }
};

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

// One red-black half-sweep (colour col) on plane p over the tile region of
// halo h around the interior, in place on `yp`; ym / ypl are planes p -/+ 1.
// `zero_start`: the plane still holds the zero initial guess (first
// half-sweep of a pre-smoother), so y = c * rhs.
template <int H, int TY, int EXW, int EXH>
__device__ __forceinline__ void rb_stage(float* yp, const float* ym, const float* ypl, const float* rp, int h, int col,
                                         int p, int X0, int Y0, int n, float cp, float ih2, bool zero_start,
                                         int tid, int nt) {
  using PL = Plane<EXW, EXH>;
  const int rw = kTX + 2 * h, rh = TY + 2 * h, half = rw / 2;
  for (int t = tid; t < half * rh; t += nt) {
    const int r = t / half, q = t - r * half;
    const int ly = H - h + r, gy = Y0 - H + ly;
    const int lx0 = H - h + 2 * q, gx0 = X0 - H + lx0;
    const int par = ((gx0 + gy + p) ^ col) & 1;
    const int lx = lx0 + par, gx = gx0 + par;
    if (gx < 1 || gx >= n || gy < 1 || gy >= n) continue;
    const int c = PL::at(lx, ly);
    float v;
    if (zero_start) {
      v = cp * rp[c];
    } else {
      const float yc = yp[c];
      float a = 6.0f * yc;
      a = a - yp[PL::at(lx - 1, ly)];
      a = a - yp[PL::at(lx + 1, ly)];
      a = a - yp[PL::at(lx, ly - 1)];
      a = a - yp[PL::at(lx, ly + 1)];
      a = a - ym[c];
      a = a - ypl[c];
      a = a * ih2;
      const float rr = rp[c] - a;
      v = yc + cp * rr;
    }
    yp[c] = v;
  }
}

// =========================================================== down-smoothing
// y'_l = Q(S^nu1(0; g_l)): S = 2 nu1 half-sweeps from zero (red first).
//
// Register columns: each thread owns K pairs of adjacent x-columns of the
// tile (with halo H = S - 1: the first half-sweep is pointwise) and keeps,
// per column, the y values of planes j-S-1 .. j and the right-hand side of
// planes j-S .. j in registers.  At step j stage s updates plane j - s;
// within a pair exactly one column has the stage's colour on that plane,
// and which one alternates with j.  The z-neighbours come from the
// column's own registers; the four in-plane neighbours come from LDS,
// where stage s publishes its updated values (double-buffered by step
// parity) for stage s + 1 to read at the next step.  One barrier per step.
template <int S, int TY, int NT>
__global__ void __launch_bounds__(NT) k_down_smooth(SecRef G, SecRef Y, Geom g, float cp, float ih2, int TZ) {
  constexpr int H = S - 1;
  constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H;
  constexpr int PW = EXW / 2, NPAIR = PW * EXH, K = (NPAIR + NT - 1) / NT;
  constexpr int LW = EXW + 2, LPL = LW * (EXH + 2);  // LDS plane with a margin of one
  constexpr int NB = S > 1 ? S - 1 : 1;
  __shared__ float pub[2][NB][LPL];
  __shared__ float outb[2][TY * kTX];
  const int tid = threadIdx.x, lane = tid & 63;
  const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * TY, Z0 = blockIdx.z * TZ;
  const int n = g.n;
  const int64_t zstride = static_cast<int64_t>(1) << (2 * g.level);

  // per-pair constants
  int pos[K];        // LDS position of column 0 of the pair
  int par[K];        // column active at step j: (par + j) & 1
  int64_t xy[K][2];  // flat x-y index of each column (or -1 outside the level)
  unsigned upd[K];   // bit (2 (s-1) + c): stage s updates column c
  unsigned outm[K];  // bit c: column c lies in the output interior; bit 2: pair exists
  int oidx[K];       // output buffer index of column 0
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = tid + k * NT;
    const bool valid = q < NPAIR;
    const int ly = valid ? q / PW : 0, lx0 = valid ? 2 * (q - ly * PW) : 0;
    const int gx0 = X0 - H + lx0, gy = Y0 - H + ly;
    pos[k] = (ly + 1) * LW + lx0 + 1;
    par[k] = (gx0 + gy - 1) & 1;
    upd[k] = 0u;
    outm[k] = 0u;
    oidx[k] = (ly - H) * kTX + (lx0 - H);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int lx = lx0 + c, gx = gx0 + c;
      const bool dom = valid && gx >= 0 && gx < n && gy >= 0 && gy < n;
      xy[k][c] = dom ? ((static_cast<int64_t>(gy) << g.level) | gx) : -1;
      const int dx = max(max(H - lx, lx - (H + kTX - 1)), 0);
      const int dy = max(max(H - ly, ly - (H + TY - 1)), 0);
      const int d = max(dx, dy);
      const bool inner = valid && gx >= 1 && gx < n && gy >= 1 && gy < n;
#pragma unroll
      for (int s = 1; s <= S; ++s)
        if (inner && d <= S - s) upd[k] |= 1u << (2 * (s - 1) + c);
      if (valid && d == 0) outm[k] |= 1u << c;
    }
    if (valid) outm[k] |= 4u;
  }
  // pairs k whose whole wave lies beyond the tile do no work
  auto wave_has = [&](int k) { return k * NT + (tid & ~63) < NPAIR; };
  float y[K][2][S + 2];
  float r[K][2][S + 1];
  RawCode pre[K][2];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int i = 0; i < S + 2; ++i) y[k][c][i] = 0.0f;
#pragma unroll
      for (int i = 0; i < S + 1; ++i) r[k][c][i] = 0.0f;
    }
  auto fetch = [&](int jj) {
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        pre[k][c] = raw_none();
        if (xy[k][c] >= 0 && jj >= 0 && jj < n) pre[k][c] = raw_load(G, jj * zstride + xy[k][c]);
      }
  };
  auto quantise_out = [&](int po, int slot) {
    if (po < Z0 || po >= Z0 + TZ) return;
    for (int rr = tid >> 6; rr < TY; rr += NT / 64) {
      const float v = outb[slot][rr * kTX + lane];
      const int64_t base = flat(g, X0, Y0 + rr, po);
      int e;
      const int32_t m = quantise_lane_f32(v, Y.B, Y.w, lane, &e);
      store_codes_wave(Y, base, lane, m, Y.n);
      if ((lane & (Y.B - 1)) == 0) Y.exps[blk(Y, base + lane)] = static_cast<int16_t>(e);
    }
  };

  const int jbeg = Z0 - S, jend = Z0 + TZ + S;
  fetch(jbeg);
  for (int j = jbeg; j < jend; ++j) {
    quantise_out(j - 1 - S, (j - 1) & 1);  // plane finished at the previous step
    // new plane j: y = 0, rhs from the prefetch
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int i = 0; i < S + 1; ++i) y[k][c][i] = y[k][c][i + 1];
        y[k][c][S + 1] = 0.0f;
#pragma unroll
        for (int i = 0; i < S; ++i) r[k][c][i] = r[k][c][i + 1];
        const int64_t idx = xy[k][c] >= 0 ? j * zstride + xy[k][c] : 0;
        r[k][c][S] = static_cast<float>(raw_value(G, idx, pre[k][c]));
      }
    if (j + 1 < jend) fetch(j + 1);
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int p = j - s;
      if (p < max(1, Z0 - (S - s)) || p > min(n - 1, Z0 + TZ + (S - s) - 1)) continue;
      const int iy = S + 1 - s;
      const float* src = pub[(j - 1) & 1][s >= 2 ? s - 2 : 0];
      float* dst = pub[j & 1][s - 1 < NB ? s - 1 : 0];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!wave_has(k)) continue;
        const int ca = (par[k] + j) & 1;
        const float yc = ca ? y[k][1][iy] : y[k][0][iy];
        const float rhs = ca ? r[k][1][S - s] : r[k][0][S - s];
        const int pa = pos[k] + ca;
        float v;
        if (s == 1) {
          v = cp * rhs;
        } else {
          const float zm = ca ? y[k][1][iy - 1] : y[k][0][iy - 1];
          const float zp = ca ? y[k][1][iy + 1] : y[k][0][iy + 1];
          float a = 6.0f * yc;
          a = a - src[pa - 1];
          a = a - src[pa + 1];
          a = a - src[pa - LW];
          a = a - src[pa + LW];
          a = a - zm;
          a = a - zp;
          a = a * ih2;
          const float rr = rhs - a;
          v = yc + cp * rr;
        }
        const bool u = (upd[k] >> (2 * (s - 1) + ca)) & 1u;
        const float yv = u ? v : yc;
        y[k][0][iy] = ca == 0 ? yv : y[k][0][iy];
        y[k][1][iy] = ca == 1 ? yv : y[k][1][iy];
        if (s < S && (outm[k] & 4u)) dst[pa] = yv;
      }
    }
    const int po = j - S;  // plane complete: both colours have their last update
    if (po >= Z0 && po < Z0 + TZ) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (outm[k] & 1u) outb[j & 1][oidx[k]] = y[k][0][1];
        if (outm[k] & 2u) outb[j & 1][oidx[k] + 1] = y[k][1][1];
      }
    }
    __syncthreads();
  }
  quantise_out(jend - 1 - S, (jend - 1) & 1);
}

// ============================================================= up-smoothing
// z = P e_{l-1}; rhs = g - A z; y = S^nu2(y'_pre; rhs); Yp = Q(y);
// u'_l = Q(dec u'_l + dec Yp) (float64); e_l = dec Yp + z when eout != null.
//
// Same register-column scheme as the down-smoothing kernel, with two more
// pipeline stages in front: z of plane j is prolongated per column from a
// coarse ring in LDS and published, and at the next step the right-hand side
// of plane j - 1 needs the published in-plane z neighbours.  The
// pre-smoothed y' of a plane enters as stage 0 and is published too.
template <int S, int TY, int NT>
__global__ void __launch_bounds__(NT) k_up_smooth(const float* __restrict__ ec, SecRef G, SecRef Y, SecRef Yp,
                                                  SecRef U, float* __restrict__ eout, Geom g, Geom gc, float cp,
                                                  float ih2, int TZ) {
  constexpr int H = S + 1;
  constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H;
  constexpr int PW = EXW / 2, NPAIR = PW * EXH, K = (NPAIR + NT - 1) / NT;
  constexpr int LW = EXW + 2, LPL = LW * (EXH + 2);
  constexpr int NC = 6, CW = EXW / 2 + 3, CH = EXH / 2 + 3, CPL = CW * CH;
  constexpr int OPT = (TY * kTX + NT - 1) / NT;
  __shared__ float cs[NC * CPL];
  __shared__ float zpub[2][LPL];
  __shared__ float pub[2][S][LPL];
  __shared__ float outb[2][TY * kTX];
  const int tid = threadIdx.x, lane = tid & 63;
  const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * TY, Z0 = blockIdx.z * TZ;
  const int n = g.n;
  const int CX0 = (X0 - H) >> 1, CY0 = (Y0 - H) >> 1;
  const int64_t zstride = static_cast<int64_t>(1) << (2 * g.level);

  int pos[K], par[K], gxy[K][2];
  int64_t xy[K][2];   // flat x-y index of a column inside the level, else -1
  unsigned upd[K];    // bit 2 (s-1) + c: stage s updates column c; bits 2S + c: rhs/y0 of column c
  unsigned outm[K];   // bit c: column c in the output interior; bit 2: pair exists
  int oidx[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int q = tid + k * NT;
    const bool valid = q < NPAIR;
    const int ly = valid ? q / PW : 0, lx0 = valid ? 2 * (q - ly * PW) : 0;
    const int gx0 = X0 - H + lx0, gy = Y0 - H + ly;
    pos[k] = (ly + 1) * LW + lx0 + 1;
    par[k] = (gx0 + gy - 1) & 1;
    upd[k] = 0u;
    outm[k] = valid ? 4u : 0u;
    oidx[k] = (ly - H) * kTX + (lx0 - H);
    gxy[k][0] = gx0;
    gxy[k][1] = gy;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int lx = lx0 + c, gx = gx0 + c;
      const bool dom = valid && gx >= 0 && gx < n && gy >= 0 && gy < n;
      xy[k][c] = dom ? ((static_cast<int64_t>(gy) << g.level) | gx) : -1;
      const int d = max(max(max(H - lx, lx - (H + kTX - 1)), 0), max(max(H - ly, ly - (H + TY - 1)), 0));
      const bool inner = valid && gx >= 1 && gx < n && gy >= 1 && gy < n;
#pragma unroll
      for (int s = 1; s <= S; ++s)
        if (inner && d <= S - s) upd[k] |= 1u << (2 * (s - 1) + c);
      if (inner && d <= S) upd[k] |= 1u << (2 * S + c);
      if (valid && d == 0) outm[k] |= 1u << c;
    }
  }
  auto wave_has = [&](int k) { return k * NT + (tid & ~63) < NPAIR; };

  float z[K][2][3];      // z of planes j-2, j-1, j
  float r[K][2][S + 1];  // rhs of planes j-1-S .. j-1
  float y[K][2][S + 2];  // y of planes j-2-S .. j-1
  RawCode gpre[K][2], ypre[K][2], upre[OPT];
  CoarseFetch<float, CW, CH, NT> cpf;
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
      for (int i = 0; i < 3; ++i) z[k][c][i] = 0.0f;
#pragma unroll
      for (int i = 0; i < S + 1; ++i) r[k][c][i] = 0.0f;
#pragma unroll
      for (int i = 0; i < S + 2; ++i) y[k][c][i] = 0.0f;
    }
  auto fetch_gy = [&](int p) {  // g and y' of plane p for the own columns
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        gpre[k][c] = raw_none();
        ypre[k][c] = raw_none();
        if (xy[k][c] >= 0 && p >= 1 && p < n && ((upd[k] >> (2 * S + c)) & 1u)) {
          const int64_t idx = p * zstride + xy[k][c];
          gpre[k][c] = raw_load(G, idx);
          ypre[k][c] = raw_load(Y, idx);
        }
      }
  };
  auto fetch_u = [&](int po) {
#pragma unroll
    for (int t = 0; t < OPT; ++t) {
      const int rr = (tid >> 6) + t * (NT / 64);
      upre[t] = raw_none();
      if (rr < TY && po >= Z0 && po < Z0 + TZ) upre[t] = raw_load(U, flat(g, X0 + lane, Y0 + rr, po));
    }
  };
  auto finish_out = [&](int po, int slot) {  // quantise y', correct u', write e
    if (po < Z0 || po >= Z0 + TZ) return;
#pragma unroll
    for (int t = 0; t < OPT; ++t) {
      const int rr = (tid >> 6) + t * (NT / 64);
      if (rr >= TY) continue;
      const float v = outb[slot][rr * kTX + lane];
      const int64_t base = flat(g, X0, Y0 + rr, po);
      const int64_t i = base + lane;
      int ey;
      const int32_t my = quantise_lane_f32(v, Yp.B, Yp.w, lane, &ey);
      store_codes_wave(Yp, base, lane, my, Yp.n);
      if ((lane & (Yp.B - 1)) == 0) Yp.exps[blk(Yp, i)] = static_cast<int16_t>(ey);
      const double dy = ey == kZeroExp ? 0.0 : ldexp(static_cast<double>(my), ey - (Yp.w - 1));
      const double vu = raw_value(U, i, upre[t]) + dy;
      int eu;
      const int64_t mu = quantise_lane(vu, U.B, U.w, &eu);
      store_codes_wave(U, base, lane, mu, U.n);
      if ((lane & (U.B - 1)) == 0) U.exps[blk(U, i)] = static_cast<int16_t>(eu);
      if (eout != nullptr) {
        const float zz = prolong_lds<float, NC, CW, CPL>(cs, CX0, CY0, X0 + lane, Y0 + rr, po);
        eout[i] = static_cast<float>(dy) + zz;
      }
    }
  };

  const int jbeg = Z0 - S - 1, jend = Z0 + TZ + S + 1;
  cpf.fetch(ec, gc, CX0, CY0, jbeg >> 1, tid);
  cpf.store(cs + ring(jbeg >> 1, NC) * CPL, tid);
  cpf.fetch(ec, gc, CX0, CY0, (jbeg >> 1) + 1, tid);
  cpf.store(cs + ring((jbeg >> 1) + 1, NC) * CPL, tid);
  fetch_gy(jbeg - 1);
  fetch_u(jbeg - 2 - S);
  __syncthreads();
  for (int j = jbeg; j < jend; ++j) {
    finish_out(j - 2 - S, (j - 1) & 1);  // plane completed at the previous step
    fetch_u(j - 1 - S);
    const bool need_c = ((j + 1) & 1) && j + 1 < jend;  // z(j+1) needs coarse plane (j+2)/2
    if (need_c) cpf.fetch(ec, gc, CX0, CY0, (j + 2) >> 1, tid);
    // (b) z of plane j for the own columns, published
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!wave_has(k)) continue;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        z[k][c][0] = z[k][c][1];
        z[k][c][1] = z[k][c][2];
        const int gx = gxy[k][0] + c, gy = gxy[k][1];
        float zz = 0.0f;
        if ((outm[k] & 4u) && j >= 0 && gx >= 0 && gy >= 0)
          zz = prolong_lds<float, NC, CW, CPL>(cs, CX0, CY0, gx, gy, j);
        z[k][c][2] = zz;
        if (outm[k] & 4u) zpub[j & 1][pos[k] + c] = zz;
      }
    }
    // (c) plane j - 1: rhs = g - A z and y0 for both columns; y0 published as stage 0
    {
      const int p = j - 1;
      const float* zs = zpub[(j - 1) & 1];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!wave_has(k)) continue;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
          for (int i = 0; i < S; ++i) r[k][c][i] = r[k][c][i + 1];
#pragma unroll
          for (int i = 0; i < S + 1; ++i) y[k][c][i] = y[k][c][i + 1];
          float rv = 0.0f, yv = 0.0f;
          if (((upd[k] >> (2 * S + c)) & 1u) && p >= 1 && p < n) {
            const int pc = pos[k] + c;
            float a = 6.0f * z[k][c][1];
            a = a - zs[pc - 1];
            a = a - zs[pc + 1];
            a = a - zs[pc - LW];
            a = a - zs[pc + LW];
            a = a - z[k][c][0];
            a = a - z[k][c][2];
            a = a * ih2;
            const int64_t idx = p * zstride + xy[k][c];
            rv = static_cast<float>(raw_value(G, idx, gpre[k][c])) - a;
            yv = static_cast<float>(raw_value(Y, idx, ypre[k][c]));
          }
          r[k][c][S] = rv;
          y[k][c][S + 1] = yv;
          if (outm[k] & 4u) pub[j & 1][0][pos[k] + c] = yv;
        }
      }
      if (j + 1 < jend) fetch_gy(j);
    }
    // (d) post-smoothing: stage s on plane j - 1 - s
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int p = j - 1 - s;
      if (p < max(1, Z0 - (S - s)) || p > min(n - 1, Z0 + TZ + (S - s) - 1)) continue;
      const int iy = S + 1 - s;
      const float* src = pub[(j - 1) & 1][s - 1];
      float* dst = pub[j & 1][s < S ? s : 0];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!wave_has(k)) continue;
        const int ca = (par[k] + j - 1) & 1;
        const float yc = ca ? y[k][1][iy] : y[k][0][iy];
        const float zm = ca ? y[k][1][iy - 1] : y[k][0][iy - 1];
        const float zp = ca ? y[k][1][iy + 1] : y[k][0][iy + 1];
        const float rhs = ca ? r[k][1][S - s] : r[k][0][S - s];
        const int pa = pos[k] + ca;
        float a = 6.0f * yc;
        a = a - src[pa - 1];
        a = a - src[pa + 1];
        a = a - src[pa - LW];
        a = a - src[pa + LW];
        a = a - zm;
        a = a - zp;
        a = a * ih2;
        const float rr = rhs - a;
        const float v = yc + cp * rr;
        const bool u = (upd[k] >> (2 * (s - 1) + ca)) & 1u;
        const float yv = u ? v : yc;
        y[k][0][iy] = ca == 0 ? yv : y[k][0][iy];
        y[k][1][iy] = ca == 1 ? yv : y[k][1][iy];
        if (s < S && (outm[k] & 4u)) dst[pa] = yv;
      }
    }
    // (e) plane j - 1 - S is complete
    const int po = j - 1 - S;
    if (po >= Z0 && po < Z0 + TZ) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (outm[k] & 1u) outb[j & 1][oidx[k]] = y[k][0][1];
        if (outm[k] & 2u) outb[j & 1][oidx[k] + 1] = y[k][1][1];
      }
    }
    if (need_c) cpf.store(cs + ring((j + 2) >> 1, NC) * CPL, tid);
    __syncthreads();
  }
  finish_out(jend - 2 - S, (jend - 1) & 1);
}

// ======================================================== residual-restrict
// g_{l-1} = Q(R(g_l - A y'_l)) on a coarse tile of 64 x CTY nodes; the fine
// level is marched plane by plane.
template <int CTY, int NT>
__global__ void __launch_bounds__(NT) k_resid_restrict(SecRef G, SecRef Y, SecRef Gc, Geom g, Geom gc, float ih2,
                                                       int TZc) {
  constexpr int YW = 2 * kTX + 4, YH = 2 * CTY + 3;  // y' tile: fine x in [2CX0-2, 2CX0+130)
  constexpr int TW = 2 * kTX + 2, TH = 2 * CTY + 1;  // t tile: fine x in [2CX0-1, 2CX0+129)
  constexpr int YPT = (YW * YH + NT - 1) / NT, GPT = (TW * TH + NT - 1) / NT;
  __shared__ float yv[3 * YW * YH];
  __shared__ float gv[2 * TW * TH];
  __shared__ float tv[3 * TW * TH];
  const int tid = threadIdx.x;
  const int CX0 = blockIdx.x * kTX, CY0 = blockIdx.y * CTY, CZ0 = blockIdx.z * TZc;
  const int n = g.n;
  const int FX0 = 2 * CX0 - 2, FY0 = 2 * CY0 - 2;  // origin of the y' tile
  RawCode ypre[YPT], gpre[GPT];
  auto fetch = [&](int q) {
#pragma unroll
    for (int k = 0; k < YPT; ++k) {
      const int t = tid + k * NT;
      const int ly = t / YW, lx = t - ly * YW;
      const int gx = FX0 + lx, gy = FY0 + ly;
      ypre[k] = raw_none();
      if (t < YW * YH && q >= 0 && q < n && gx >= 0 && gx < n && gy >= 0 && gy < n)
        ypre[k] = raw_load(Y, flat(g, gx, gy, q));
    }
#pragma unroll
    for (int k = 0; k < GPT; ++k) {
      const int t = tid + k * NT;
      const int ly = t / TW, lx = t - ly * TW;
      const int gx = FX0 + 1 + lx, gy = FY0 + 1 + ly;
      gpre[k] = raw_none();
      if (t < TW * TH && q >= 0 && q < n && gx >= 0 && gx < n && gy >= 0 && gy < n)
        gpre[k] = raw_load(G, flat(g, gx, gy, q));
    }
  };
  const int qend = 2 * (CZ0 + TZc);
  fetch(2 * CZ0 - 2);
  for (int q = 2 * CZ0 - 2; q <= qend; ++q) {
    {  // y'(q) and g(q) from the prefetch
      float* yp = yv + ring(q, 3) * YW * YH;
#pragma unroll
      for (int k = 0; k < YPT; ++k) {
        const int t = tid + k * NT;
        if (t >= YW * YH) continue;
        const int ly = t / YW, lx = t - ly * YW;
        const int gx = FX0 + lx, gy = FY0 + ly;
        const int64_t idx = (gx >= 0 && gy >= 0 && q >= 0) ? flat(g, gx, gy, q) : 0;
        yp[t] = static_cast<float>(raw_value(Y, idx, ypre[k]));
      }
      float* gp = gv + ring(q, 2) * TW * TH;
#pragma unroll
      for (int k = 0; k < GPT; ++k) {
        const int t = tid + k * NT;
        if (t >= TW * TH) continue;
        const int ly = t / TW, lx = t - ly * TW;
        const int gx = FX0 + 1 + lx, gy = FY0 + 1 + ly;
        const int64_t idx = (gx >= 0 && gy >= 0 && q >= 0) ? flat(g, gx, gy, q) : 0;
        gp[t] = static_cast<float>(raw_value(G, idx, gpre[k]));
      }
    }
    if (q + 1 <= qend) fetch(q + 1);
    __syncthreads();
    const int p = q - 1;  // t on plane p
    if (p >= 2 * CZ0 - 1) {
      const float* yc = yv + ring(p, 3) * YW * YH;
      const float* ym = yv + ring(p - 1, 3) * YW * YH;
      const float* ypl = yv + ring(p + 1, 3) * YW * YH;
      const float* gp = gv + ring(p, 2) * TW * TH;
      float* tp = tv + ring(p, 3) * TW * TH;
      for (int t = tid; t < TW * TH; t += NT) {
        const int ly = t / TW, lx = t - ly * TW;
        const int gx = FX0 + 1 + lx, gy = FY0 + 1 + ly;
        float v = 0.0f;
        if (p >= 1 && p < n && gx >= 1 && gx < n && gy >= 1 && gy < n) {
          const int c = (ly + 1) * YW + (lx + 1);
          float a = 6.0f * yc[c];
          a = a - yc[c - 1];
          a = a - yc[c + 1];
          a = a - yc[c - YW];
          a = a - yc[c + YW];
          a = a - ym[c];
          a = a - ypl[c];
          a = a * ih2;
          v = gp[t] - a;
        }
        tp[t] = v;
      }
    }
    __syncthreads();
    if ((q & 1) == 0) {  // coarse plane K = q/2 - 1 has t on 2K-1 .. 2K+1
      const int K = q / 2 - 1;
      if (K >= CZ0 && K < CZ0 + TZc) {
        const int lane = tid & 63;
        for (int r = tid >> 6; r < CTY; r += NT / 64) {
          const int I = CX0 + lane, J = CY0 + r;
          float s = 0.0f;
          if (I >= 1 && J >= 1 && K >= 1) {
            bool first = true;
            for (int oz = -1; oz <= 1; ++oz) {
              const double wz = oz == 0 ? 0.5 : 0.25;
              const float* tp = tv + ring(2 * K + oz, 3) * TW * TH;
              for (int oy = -1; oy <= 1; ++oy) {
                const double wy = oy == 0 ? 0.5 : 0.25;
                for (int ox = -1; ox <= 1; ++ox) {
                  const double wx = ox == 0 ? 0.5 : 0.25;
                  const int lx = 2 * I + ox - (FX0 + 1), ly = 2 * J + oy - (FY0 + 1);
                  const float t = static_cast<float>(wz * wy * wx) * tp[ly * TW + lx];
                  s = first ? t : s + t;
                  first = false;
                }
              }
            }
          }
          const int64_t base = flat(gc, CX0, J, K);
          int e;
          const int32_t m = quantise_lane_f32(s, Gc.B, Gc.w, lane, &e);
          store_codes_wave(Gc, base, lane, m, Gc.n);
          if ((lane & (Gc.B - 1)) == 0) Gc.exps[blk(Gc, base + lane)] = static_cast<int16_t>(e);
        }
      }
    }
  }
}

// ============================================================= IR residual
// g_Lp = Q(f - A(dec u'_Lp + P u_{Lp-1})) in float64 (Alg. 2 on the finest
// level of the current FMG level); f is the caller's full node array of the
// finest level L, sampled with stride 2^(L - Lp).
template <int TY, int NT>
__global__ void __launch_bounds__(NT) k_ir_residual(SecRef U, const double* __restrict__ uc,
                                                    const double* __restrict__ f, int Lfull, Geom g, Geom gc,
                                                    double ih2, SecRef Gout, int TZ, int* nonfinite,
                                                    double* sumsq) {
  constexpr int EXW = kTX + 2, EXH = TY + 2, PLS = EXW * EXH;
  constexpr int NC = 3, CW = EXW / 2 + 3, CH = EXH / 2 + 3, CPL = CW * CH;
  constexpr int UPT = (PLS + NT - 1) / NT, FPT = (TY * 64 + NT - 1) / NT;
  __shared__ double us[3 * PLS];
  __shared__ double cs[NC * CPL];
  const int tid = threadIdx.x, lane = tid & 63;
  const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * TY, Z0 = blockIdx.z * TZ;
  const int n = g.n;
  const int CX0 = (X0 - 1) >> 1, CY0 = (Y0 - 1) >> 1;
  const int64_t N = (static_cast<int64_t>(1) << Lfull) + 1;
  const int st = 1 << (Lfull - g.level);
  const int jbeg = Z0 - 1, jend = Z0 + TZ + 1;
  CoarseFetch<double, CW, CH, NT> cpf;
  RawCode upre[UPT];
  double fpre[FPT];
  auto fetch_u = [&](int jj) {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int t = tid + k * NT;
      const int ly = t / EXW, lx = t - ly * EXW;
      const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
      upre[k] = raw_none();
      if (t < PLS && jj >= 0 && jj < n && gx >= 0 && gx < n && gy >= 0 && gy < n)
        upre[k] = raw_load(U, flat(g, gx, gy, jj));
    }
  };
  auto fetch_f = [&](int p) {  // f at the output rows of plane p
#pragma unroll
    for (int k = 0; k < FPT; ++k) {
      const int r = (tid >> 6) + k * (NT / 64);
      const int gx = X0 + lane, gy = Y0 + r;
      fpre[k] = 0.0;
      if (r < TY && p >= 1 && p < n && gx >= 1 && gy >= 1)
        fpre[k] = f[(static_cast<int64_t>(p) * st * N + static_cast<int64_t>(gy) * st) * N +
                    static_cast<int64_t>(gx) * st];
    }
  };
  cpf.fetch(uc, gc, CX0, CY0, jbeg >> 1, tid);
  cpf.store(cs + ring(jbeg >> 1, NC) * CPL, tid);
  cpf.fetch(uc, gc, CX0, CY0, (jbeg >> 1) + 1, tid);
  cpf.store(cs + ring((jbeg >> 1) + 1, NC) * CPL, tid);
  fetch_u(jbeg);
  fetch_f(jbeg - 1);
  for (int j = jbeg; j < jend; ++j) {
    if (j != jbeg && (j & 1)) cpf.store(cs + ring((j + 1) >> 1, NC) * CPL, tid);
    __syncthreads();
    {  // decoded solution on plane j (tile plus a halo of one)
      double* up = us + ring(j, 3) * PLS;
#pragma unroll
      for (int k = 0; k < UPT; ++k) {
        const int t = tid + k * NT;
        if (t >= PLS) continue;
        const int ly = t / EXW, lx = t - ly * EXW;
        const int gx = X0 - 1 + lx, gy = Y0 - 1 + ly;
        double v = 0.0;
        if (j >= 0 && j < n && gx >= 0 && gx < n && gy >= 0 && gy < n)
          v = raw_value(U, flat(g, gx, gy, j), upre[k]) + prolong_lds<double, NC, CW, CPL>(cs, CX0, CY0, gx, gy, j);
        up[t] = v;
      }
      if (j + 1 < jend) {
        fetch_u(j + 1);
        if ((j + 1) & 1) cpf.fetch(uc, gc, CX0, CY0, (j + 2) >> 1, tid);
      }
    }
    __syncthreads();
    const int p = j - 1;
    if (p >= Z0 && p < Z0 + TZ) {
      const double* uc0 = us + ring(p, 3) * PLS;
      const double* um = us + ring(p - 1, 3) * PLS;
      const double* upl = us + ring(p + 1, 3) * PLS;
#pragma unroll
      for (int k = 0; k < FPT; ++k) {
        const int r = (tid >> 6) + k * (NT / 64);
        if (r >= TY) continue;
        const int gx = X0 + lane, gy = Y0 + r;
        double t = 0.0;
        if (p >= 1 && gx >= 1 && gy >= 1) {
          const int c = (r + 1) * EXW + lane + 1;
          double a = 6.0 * uc0[c];
          a = a - uc0[c - 1];
          a = a - uc0[c + 1];
          a = a - uc0[c - EXW];
          a = a - uc0[c + EXW];
          a = a - um[c];
          a = a - upl[c];
          a = a * ih2;
          t = fpre[k] - a;
        }
        if (nonfinite != nullptr && !isfinite(t)) atomicOr(nonfinite, 1);
        if (sumsq != nullptr) {
          double a2 = t * t;
          for (int off = 32; off > 0; off >>= 1) a2 += __shfl_xor(a2, off, 64);
          if (lane == 0) atomicAdd(sumsq, a2);
        }
        const int64_t base = flat(g, X0, gy, p);
        int e;
        const int64_t m = quantise_lane(t, Gout.B, Gout.w, &e);
        store_codes_wave(Gout, base, lane, m, Gout.n);
        if ((lane & (Gout.B - 1)) == 0) Gout.exps[blk(Gout, base + lane)] = static_cast<int16_t>(e);
      }
    }
    fetch_f(j);
  }
}

// ============================================================ final decode
// u (full node grid of level g) = dec u'_l + P u_{l-1}; far boundary 0.
__global__ void __launch_bounds__(256) k_decode_full(SecRef U, const double* __restrict__ uc, Geom g, Geom gc,
                                                     double* __restrict__ full) {
  const int64_t N = g.n + 1;
  const int64_t total = N * N * N;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (idx >= total) return;
  const int i = static_cast<int>(idx % N);
  const int j = static_cast<int>((idx / N) % N);
  const int k = static_cast<int>(idx / (N * N));
  double v = 0.0;
  if (i < g.n && j < g.n && k < g.n) {
    const int ti = i >> 1, tj = j >> 1, tk = k >> 1;
    const int pi = i & 1, pj = j & 1, pk = k & 1;
    double s = 0.0;
    bool first = true;
    for (int oz = 0; oz <= pk; ++oz)
      for (int oy = 0; oy <= pj; ++oy)
        for (int ox = 0; ox <= pi; ++ox) {
          const double w = (pk ? 0.5 : 1.0) * (pj ? 0.5 : 1.0) * (pi ? 0.5 : 1.0);
          const double t = w * at(uc, gc, ti + ox, tj + oy, tk + oz);
          s = first ? t : s + t;
          first = false;
        }
    v = decode_value(U, flat(g, i, j, k)) + s;
  }
  full[idx] = v;
}

// =============================================================== launchers
static int pick_tz(int n, int tiles_xy, int min_tz) {
  int tz = n;
  while (tz > min_tz && static_cast<int64_t>(tiles_xy) * (n / tz) < 2048) tz >>= 1;
  return tz;
}

static double sec_b(const SecRef& s) {
  const double nb = static_cast<double>((s.n + s.B - 1) / s.B);
  return nb * s.B * s.cbits / 8.0 + 2.0 * nb;
}

#define CMG_FLAUNCH(name, nbytes, kernel, grid, block, stream, ...)                        \
  do {                                                                                    \
    if (g_timing != nullptr) g_timing->begin((name), static_cast<double>(nbytes), stream); \
    hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                      \
    if (g_timing != nullptr) g_timing->end(stream);                                       \
  } while (0)

constexpr int kDownTY = 16, kUpTY = 16, kResTY = 16, kRRCTY = 4, kUpNT = 512;

bool fused_down_smooth(const SecRef& G, const SecRef& Y, const Geom& g, int nu, float cp, float ih2,
                       hipStream_t st) {
  if (g.dim != 3 || g.n < kTX) return false;
  const int ty = kDownTY;
  const int tz = pick_tz(g.n, (g.n / kTX) * (g.n / ty), 16);
  const dim3 grid(g.n / kTX, g.n / ty, g.n / tz);
  const double bytes = sec_b(G) + sec_b(Y);
  if (nu == 2)
    CMG_FLAUNCH("k_down_smooth<4>", bytes, (k_down_smooth<4, kDownTY, 256>), grid, dim3(256), st, G, Y, g, cp, ih2,
                tz);
  else if (nu == 1)
    CMG_FLAUNCH("k_down_smooth<2>", bytes, (k_down_smooth<2, kDownTY, 256>), grid, dim3(256), st, G, Y, g, cp, ih2,
                tz);
  else
    return false;
  return true;
}

bool fused_up_smooth(const float* ec, const SecRef& G, const SecRef& Y, const SecRef& Yp, const SecRef& U,
                     float* eout, const Geom& g, const Geom& gc, int nu, float cp, float ih2, hipStream_t st) {
  if (g.dim != 3 || g.n < kTX) return false;
  const int ty = kUpTY;
  const int tz = pick_tz(g.n, (g.n / kTX) * (g.n / ty), 16);
  const dim3 grid(g.n / kTX, g.n / ty, g.n / tz);
  const double bytes = sec_b(G) + sec_b(Y) + sec_b(Yp) + 2.0 * sec_b(U) + 4.0 * gc.size + (eout ? 4.0 * g.size : 0.0);
  if (nu == 2)
    CMG_FLAUNCH("k_up_smooth<4>", bytes, (k_up_smooth<4, kUpTY, kUpNT>), grid, dim3(kUpNT), st, ec, G, Y, Yp, U, eout, g,
                gc, cp, ih2, tz);
  else if (nu == 1)
    CMG_FLAUNCH("k_up_smooth<2>", bytes, (k_up_smooth<2, kUpTY, kUpNT>), grid, dim3(kUpNT), st, ec, G, Y, Yp, U, eout, g,
                gc, cp, ih2, tz);
  else
    return false;
  return true;
}

bool fused_resid_restrict(const SecRef& G, const SecRef& Y, const SecRef& Gc, const Geom& g, const Geom& gc,
                          float ih2, hipStream_t st) {
  if (g.dim != 3 || gc.n < kTX) return false;
  const int tz = pick_tz(gc.n, (gc.n / kTX) * (gc.n / kRRCTY), 8);
  const dim3 grid(gc.n / kTX, gc.n / kRRCTY, gc.n / tz);
  const double bytes = sec_b(G) + sec_b(Y) + sec_b(Gc);
  CMG_FLAUNCH("k_resid_restrict", bytes, (k_resid_restrict<kRRCTY, 256>), grid, dim3(256), st, G, Y, Gc, g, gc, ih2,
              tz);
  return true;
}

bool fused_ir_residual(const SecRef& U, const double* uc, const double* f, int Lfull, const Geom& g, const Geom& gc,
                       double ih2, const SecRef& Gout, int* nonfinite, double* sumsq, hipStream_t st) {
  if (g.dim != 3 || g.n < kTX) return false;
  const int ty = kResTY;
  const int tz = pick_tz(g.n, (g.n / kTX) * (g.n / ty), 16);
  const dim3 grid(g.n / kTX, g.n / ty, g.n / tz);
  const double bytes = sec_b(U) + 8.0 * gc.size + 8.0 * g.size + sec_b(Gout);
  CMG_FLAUNCH("k_ir_residual", bytes, (k_ir_residual<kResTY, 256>), grid, dim3(256), st, U, uc, f, Lfull, g, gc, ih2,
              Gout, tz, nonfinite, sumsq);
  return true;
}

void launch_decode_full(const SecRef& U, const double* uc, const Geom& g, const Geom& gc, double* full,
                        hipStream_t st) {
  const int64_t N = g.n + 1;
  const int64_t total = N * N * N;
  CMG_FLAUNCH("k_decode_full", sec_b(U) + 8.0 * gc.size + 8.0 * total, k_decode_full,
              dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), st, U, uc, g, gc, full);
}

}  // namespace cmg
