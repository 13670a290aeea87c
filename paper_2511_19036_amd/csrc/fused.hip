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
template <int S, int TY, int NT>
__global__ void __launch_bounds__(NT) k_down_smooth(SecRef G, SecRef Y, Geom g, float cp, float ih2, int TZ) {
  constexpr int H = S - 1;  // the first half-sweep is pointwise
  constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H;
  using PL = Plane<EXW, EXH>;
  constexpr int NY = S + 2, NR = S + 1;
  constexpr int PPT = (PL::SIZE + NT - 1) / NT;
  __shared__ float ys[NY * PL::SIZE];
  __shared__ float rs[NR * PL::SIZE];
  const int tid = threadIdx.x;
  const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * TY, Z0 = blockIdx.z * TZ;
  const int n = g.n;
  RawCode pre[PPT];
  auto fetch = [&](int jj) {
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
      const int t = tid + k * NT;
      const int ly = t / EXW, lx = t - ly * EXW;
      const int gx = X0 - H + lx, gy = Y0 - H + ly;
      pre[k] = raw_none();
      if (t < PL::SIZE && jj >= 0 && jj < n && gx >= 0 && gx < n && gy >= 0 && gy < n)
        pre[k] = raw_load(G, flat(g, gx, gy, jj));
    }
  };
  const int jend = Z0 + TZ + S;
  fetch(Z0 - S);
  for (int j = Z0 - S; j < jend; ++j) {
    {  // plane j: decoded g (prefetched last step), zero y
      float* yp = ys + ring(j, NY) * PL::SIZE;
      float* rp = rs + ring(j, NR) * PL::SIZE;
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const int t = tid + k * NT;
        if (t < PL::SIZE) {
          const int ly = t / EXW, lx = t - ly * EXW;
          const int gx = X0 - H + lx, gy = Y0 - H + ly;
          const int64_t idx = (gx >= 0 && gy >= 0 && j >= 0) ? flat(g, gx, gy, j) : 0;
          const int c = PL::at(lx, ly);
          rp[c] = static_cast<float>(raw_value(G, idx, pre[k]));
          yp[c] = 0.0f;
        }
      }
    }
    if (j + 1 < jend) fetch(j + 1);
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int p = j - s;
      if (p >= Z0 - (S - s) && p < Z0 + TZ + (S - s) && p >= 1 && p <= n - 1)
        rb_stage<H, TY, EXW, EXH>(ys + ring(p, NY) * PL::SIZE, ys + ring(p - 1, NY) * PL::SIZE,
                                  ys + ring(p + 1, NY) * PL::SIZE, rs + ring(p, NR) * PL::SIZE, S - s, (s - 1) & 1,
                                  p, X0, Y0, n, cp, ih2, s == 1, tid, NT);
      __syncthreads();
    }
    const int po = j - S;
    if (po >= Z0 && po < Z0 + TZ) {
      const float* yp = ys + ring(po, NY) * PL::SIZE;
      const int lane = tid & 63;
      for (int r = tid >> 6; r < TY; r += NT / 64) {
        const float v = yp[PL::at(H + lane, H + r)];
        const int64_t base = flat(g, X0, Y0 + r, po);
        int e;
        const int64_t m = quantise_lane(static_cast<double>(v), Y.B, Y.w, &e);
        store_codes_wave(Y, base, lane, m, Y.n);
        if ((lane & (Y.B - 1)) == 0) Y.exps[blk(Y, base + lane)] = static_cast<int16_t>(e);
      }
    }
  }
}

// ============================================================= up-smoothing
// z = P e_{l-1}; rhs = g - A z; y = S^nu2(y'_pre; rhs); Yp = Q(y);
// u'_l = Q(dec u'_l + dec Yp) (float64); e_l = dec Yp + z when eout != null.
template <int S, int TY, int NT>
__global__ void __launch_bounds__(NT) k_up_smooth(const float* __restrict__ ec, SecRef G, SecRef Y, SecRef Yp,
                                                  SecRef U, float* __restrict__ eout, Geom g, Geom gc, float cp,
                                                  float ih2, int TZ) {
  constexpr int H = S + 1;
  constexpr int EXW = kTX + 2 * H, EXH = TY + 2 * H;
  using PL = Plane<EXW, EXH>;
  constexpr int NZ = 3, NY = S + 2, NR = S + 1;
  constexpr int NC = 6, CW = EXW / 2 + 3, CH = EXH / 2 + 3, CPL = CW * CH;
  constexpr int RW = kTX + 2 * S, RH = TY + 2 * S, RPT = (RW * RH + NT - 1) / NT;
  constexpr int OPT = (TY * 64 + NT - 1) / NT;
  __shared__ float zs[NZ * PL::SIZE];
  __shared__ float ys[NY * PL::SIZE];
  __shared__ float rs[NR * PL::SIZE];
  __shared__ float cs[NC * CPL];
  const int tid = threadIdx.x, lane = tid & 63;
  const int X0 = blockIdx.x * kTX, Y0 = blockIdx.y * TY, Z0 = blockIdx.z * TZ;
  const int n = g.n;
  const int CX0 = (X0 - H) >> 1, CY0 = (Y0 - H) >> 1;
  const int jbeg = Z0 - S - 1, jend = Z0 + TZ + S + 1;
  CoarseFetch<float, CW, CH, NT> cpf;
  RawCode gpre[RPT], ypre[RPT], upre[OPT];
  auto fetch_gy = [&](int p) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int t = tid + k * NT;
      const int ry = t / RW, rx = t - ry * RW;
      const int gx = X0 - H + rx + 1, gy = Y0 - H + ry + 1;
      gpre[k] = raw_none();
      ypre[k] = raw_none();
      if (t < RW * RH && p >= 1 && p < n && gx >= 1 && gx < n && gy >= 1 && gy < n) {
        const int64_t idx = flat(g, gx, gy, p);
        gpre[k] = raw_load(G, idx);
        ypre[k] = raw_load(Y, idx);
      }
    }
  };
  auto fetch_u = [&](int po) {
#pragma unroll
    for (int k = 0; k < OPT; ++k) {
      const int r = (tid >> 6) + k * (NT / 64);
      upre[k] = raw_none();
      if (r < TY && po >= Z0 && po < Z0 + TZ) upre[k] = raw_load(U, flat(g, X0 + lane, Y0 + r, po));
    }
  };
  // prologue: the two coarse planes of z(jbeg), g and y' of plane jbeg - 1
  cpf.fetch(ec, gc, CX0, CY0, jbeg >> 1, tid);
  cpf.store(cs + ring(jbeg >> 1, NC) * CPL, tid);
  cpf.fetch(ec, gc, CX0, CY0, (jbeg >> 1) + 1, tid);
  cpf.store(cs + ring((jbeg >> 1) + 1, NC) * CPL, tid);
  fetch_gy(jbeg - 1);
  fetch_u(jbeg - 1 - S);
  for (int j = jbeg; j < jend; ++j) {
    // (a) the coarse plane (j + 1) / 2 that z(j) needs for odd j
    if (j != jbeg && (j & 1)) cpf.store(cs + ring((j + 1) >> 1, NC) * CPL, tid);
    __syncthreads();
    {  // (b) z on plane j over the whole tile
      float* zp = zs + ring(j, NZ) * PL::SIZE;
      for (int t = tid; t < PL::SIZE; t += NT) {
        const int ly = t / EXW, lx = t - ly * EXW;
        const int gx = X0 - H + lx, gy = Y0 - H + ly;
        float z = 0.0f;
        if (j >= 0 && gx >= 0 && gy >= 0) z = prolong_lds<float, NC, CW, CPL>(cs, CX0, CY0, gx, gy, j);
        zp[PL::at(lx, ly)] = z;
      }
    }
    __syncthreads();
    {  // (c) plane j-1: rhs = g - A z and the pre-smoothed y, on halo S
      const int p = j - 1;
      float* rp = rs + ring(p, NR) * PL::SIZE;
      float* yp = ys + ring(p, NY) * PL::SIZE;
      const float* zc = zs + ring(p, NZ) * PL::SIZE;
      const float* zm = zs + ring(p - 1, NZ) * PL::SIZE;
      const float* zpl = zs + ring(p + 1, NZ) * PL::SIZE;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int t = tid + k * NT;
        if (t >= RW * RH) continue;
        const int ry = t / RW, rx = t - ry * RW;
        const int lx = rx + 1, ly = ry + 1;
        const int gx = X0 - H + lx, gy = Y0 - H + ly;
        const int c = PL::at(lx, ly);
        float r = 0.0f, y0 = 0.0f;
        if (p >= 1 && p < n && gx >= 1 && gx < n && gy >= 1 && gy < n) {
          const int64_t idx = flat(g, gx, gy, p);
          float a = 6.0f * zc[c];
          a = a - zc[PL::at(lx - 1, ly)];
          a = a - zc[PL::at(lx + 1, ly)];
          a = a - zc[PL::at(lx, ly - 1)];
          a = a - zc[PL::at(lx, ly + 1)];
          a = a - zm[c];
          a = a - zpl[c];
          a = a * ih2;
          r = static_cast<float>(raw_value(G, idx, gpre[k])) - a;
          y0 = static_cast<float>(raw_value(Y, idx, ypre[k]));
        }
        rp[c] = r;
        yp[c] = y0;
      }
      // prefetch for the next step: g and y' of plane j, coarse plane of z(j+1)
      if (j + 1 < jend) {
        fetch_gy(j);
        if ((j + 1) & 1) cpf.fetch(ec, gc, CX0, CY0, (j + 2) >> 1, tid);
      }
    }
    __syncthreads();
#pragma unroll
    for (int s = 1; s <= S; ++s) {  // (d) post-smoothing pipeline
      const int p = j - 1 - s;
      if (p >= Z0 - (S - s) && p < Z0 + TZ + (S - s) && p >= 1 && p <= n - 1)
        rb_stage<H, TY, EXW, EXH>(ys + ring(p, NY) * PL::SIZE, ys + ring(p - 1, NY) * PL::SIZE,
                                  ys + ring(p + 1, NY) * PL::SIZE, rs + ring(p, NR) * PL::SIZE, S - s, (s - 1) & 1,
                                  p, X0, Y0, n, cp, ih2, false, tid, NT);
      __syncthreads();
    }
    const int po = j - 1 - S;  // (e) output
    if (po >= Z0 && po < Z0 + TZ) {
      const float* yp = ys + ring(po, NY) * PL::SIZE;
#pragma unroll
      for (int k = 0; k < OPT; ++k) {
        const int r = (tid >> 6) + k * (NT / 64);
        if (r >= TY) continue;
        const float v = yp[PL::at(H + lane, H + r)];
        const int64_t base = flat(g, X0, Y0 + r, po);
        const int64_t i = base + lane;
        int ey;
        const int64_t my = quantise_lane(static_cast<double>(v), Yp.B, Yp.w, &ey);
        store_codes_wave(Yp, base, lane, my, Yp.n);
        if ((lane & (Yp.B - 1)) == 0) Yp.exps[blk(Yp, i)] = static_cast<int16_t>(ey);
        const double dy = ey == kZeroExp ? 0.0 : ldexp(static_cast<double>(my), ey - (Yp.w - 1));
        const double vu = raw_value(U, i, upre[k]) + dy;
        int eu;
        const int64_t mu = quantise_lane(vu, U.B, U.w, &eu);
        store_codes_wave(U, base, lane, mu, U.n);
        if ((lane & (U.B - 1)) == 0) U.exps[blk(U, i)] = static_cast<int16_t>(eu);
        if (eout != nullptr) {
          const float z = prolong_lds<float, NC, CW, CPL>(cs, CX0, CY0, X0 + lane, Y0 + r, po);
          eout[i] = static_cast<float>(dy) + z;
        }
      }
    }
    fetch_u(j - S);
  }
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
          const int64_t m = quantise_lane(static_cast<double>(s), Gc.B, Gc.w, &e);
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
