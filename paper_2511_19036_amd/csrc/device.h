// Device-side building blocks: BFP code access, level indexing, stencils.
//
// Every floating-point expression here follows a fixed evaluation order so
// that results are reproducible bit for bit (the library is compiled with
// -ffp-contract=off, i.e. no fused multiply-add):
//   * stencil neighbour terms are taken in the order -x, +x, -y, +y, -z, +z;
//   * Poisson:   (A u)_p = (2d*u_p - u_-x - u_+x - ...) * 4^l;
//   * diffusion: (A u)_p = (k_-x (u_p - u_-x) + k_+x (u_p - u_+x) + ...) * 4^l,
//     k_dir the mean of the 2^(d-1) cells sharing the edge, summed in C order
//     of the cells and then scaled by 2^-(d-1);
//   * interpolation: sum of the weighted coarse neighbours in C order;
//   * full weighting: sum over offsets -1, 0, +1 in C order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmg {

constexpr int16_t kZeroExp = -32768;

// One BFP section as a kernel argument.
struct SecRef {
  void* codes;      // container storage
  int16_t* exps;    // one exponent per block
  int64_t n;        // values (padded level size)
  int32_t B;        // block length, 32 or 64
  int32_t w;        // width of the stored codes (bits, sign included): decoding uses it
  int32_t cbits;    // container: 8, 12, 16, 32 or 64
  // Width a correction (u <- Q(dec u + dec y)) quantises the new codes to;
  // 0: w.  Widening a section to a new FMG level's width changes no value,
  // so it is left to the section's first correction on that level.
  int32_t wq = 0;
};
__host__ __device__ __forceinline__ int corr_width(const SecRef& s) { return s.wq > 0 ? s.wq : s.w; }

// ------------------------------------------------------------------ codes
// Block index of value i (B is 32 or 64: a shift, never a division).
__device__ __forceinline__ int64_t blk(const SecRef& s, int64_t i) { return i >> (s.B == 64 ? 6 : 5); }
// Values in the section's whole blocks.
__device__ __forceinline__ int64_t limit_of(const SecRef& s) {
  const int sh = s.B == 64 ? 6 : 5;
  return ((s.n + s.B - 1) >> sh) << sh;
}

__device__ __forceinline__ int64_t load_code(const SecRef& s, int64_t i) {
  switch (s.cbits) {
    case 8: return static_cast<const int8_t*>(s.codes)[i];
    case 16: return static_cast<const int16_t*>(s.codes)[i];
    case 32: return static_cast<const int32_t*>(s.codes)[i];
    case 64: return static_cast<const int64_t*>(s.codes)[i];
    default: {  // 12-bit: value i at bit 12 i
      const uint8_t* b = static_cast<const uint8_t*>(s.codes);
      int64_t byte = (i * 3) >> 1;
      uint32_t lo = b[byte], hi = b[byte + 1];
      uint32_t v = (i & 1) ? ((lo >> 4) | (hi << 4)) : (lo | ((hi & 0xFu) << 8));
      return (v & 0x800u) ? static_cast<int64_t>(v) - 4096 : static_cast<int64_t>(v);
    }
  }
}

__device__ __forceinline__ void store_code(const SecRef& s, int64_t i, int64_t m) {
  switch (s.cbits) {
    case 8: static_cast<int8_t*>(s.codes)[i] = static_cast<int8_t>(m); break;
    case 16: static_cast<int16_t*>(s.codes)[i] = static_cast<int16_t>(m); break;
    case 32: static_cast<int32_t*>(s.codes)[i] = static_cast<int32_t>(m); break;
    case 64: static_cast<int64_t*>(s.codes)[i] = m; break;
    default: break;  // 12-bit codes are written a wave at a time (store_codes_wave)
  }
}

// Exact value m * 2^(e - (w - 1)) of code i (0 for an all-zero block).
__device__ __forceinline__ double decode_value(const SecRef& s, int64_t i) {
  const int e = s.exps[blk(s, i)];
  if (e == kZeroExp) return 0.0;
  return ldexp(static_cast<double>(load_code(s, i)), e - (s.w - 1));
}

// Raw code and exponent of one value of a library-owned section: the two
// 32-bit words holding the code's bits (value i occupies bits
// [i*cbits, (i+1)*cbits) of the little-endian code stream for every
// container) and the block exponent.  No arithmetic touches the loaded
// registers here, so the loads can stay in flight across barriers until
// raw_value() consumes them; the field extraction is branch-free.  Reads up
// to 8 bytes past the value: section buffers carry 16 bytes of padding.
struct RawCode {
  uint32_t lo, hi;
  int e;
};

__device__ __forceinline__ RawCode raw_none() { return RawCode{0u, 0u, kZeroExp}; }

__device__ __forceinline__ RawCode raw_load(const SecRef& s, int64_t i) {
  const uint32_t* w = static_cast<const uint32_t*>(s.codes) + ((i * s.cbits) >> 5);
  return RawCode{w[0], w[1], s.exps[blk(s, i)]};
}

// Value of a raw code (same result as decode_value).
__device__ __forceinline__ double raw_value(const SecRef& s, int64_t i, const RawCode& r) {
  const int sh = static_cast<int>((i * s.cbits) & 31);
  const uint64_t cat = (static_cast<uint64_t>(r.hi) << 32) | r.lo;
  const int64_t m = static_cast<int64_t>(cat << (64 - sh - s.cbits)) >> (64 - s.cbits);
  const double v = ldexp(static_cast<double>(m), r.e - (s.w - 1));
  return r.e == kZeroExp ? 0.0 : v;
}

// Wave-wide max over groups of `width` lanes (width 32 or 64).
// ------------------------------------------------------- block exponents
// Block quantisation uses this fact: with E(a) the exponent that a block
// whose maximum magnitude is a receives (the frexp exponent of a, plus one
// when a rounds up to 2^(w-1) at w bits), E is non-decreasing in a, so the
// block exponent equals the largest E over the block's values.  Each lane
// computes its own E and the block takes an integer maximum over its lanes
// (DPP row reductions and readlane), which gives the same exponent and codes
// as rounding the block maximum itself.
constexpr int kNoExp = INT32_MIN;

template <int CTRL>
__device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

// Max over the lanes of each block of B = 2^LB lanes.  All 64 lanes active.
// Four DPP steps leave every lane with the maximum of its row of 16; a
// row_bcast:15 step folds row 0 into row 1 and row 2 into row 3, and for
// B = 64 a row_bcast:31 step folds lane 31 into rows 2 and 3.  The block
// maximum is then read from the block's last lane: for B = 64 the result is
// wave-uniform (a scalar register).
template <int LB>
__device__ __forceinline__ int block_max_int(int a, int lane) {
  a = max(a, dpp_int<0xB1>(a));   // quad_perm 1,0,3,2
  a = max(a, dpp_int<0x4E>(a));   // quad_perm 2,3,0,1
  a = max(a, dpp_int<0x141>(a));  // row_half_mirror
  a = max(a, dpp_int<0x140>(a));  // row_mirror
  a = max(a, __builtin_amdgcn_update_dpp(INT32_MIN, a, 0x142, 0xA, 0xF, false));  // row_bcast:15, rows 1 and 3
  if (LB == 6) {
    a = max(a, __builtin_amdgcn_update_dpp(INT32_MIN, a, 0x143, 0xC, 0xF, false));  // row_bcast:31, rows 2 and 3
    return __builtin_amdgcn_readlane(a, 63);
  }
  const int h0 = __builtin_amdgcn_readlane(a, 31), h1 = __builtin_amdgcn_readlane(a, 63);
  return lane < 32 ? h0 : h1;
}

// Per-lane exponent E(|v|) at width w (kNoExp for 0).  With frexp |v| =
// m 2^e (1/2 <= m < 1), the scaled value m 2^(w-1) rounds to 2^(w-1) at w
// bits exactly when m >= 1 - 2^-w (its tie rounds to the even 2^(w-1)), so
// E = e + [m >= lim] with lim = 1 - 2^-w, which is exact in the value's
// type for the widths used (w <= 24 in float, w <= 53 in double).
__device__ __forceinline__ float exp_lim(float, int w) { return __int_as_float(0x3F800000 - (1 << (24 - w))); }
__device__ __forceinline__ double exp_lim(double, int w) {
  return __longlong_as_double(0x3FF0000000000000LL - (1LL << (53 - w)));
}
__device__ __forceinline__ int lane_exp(float v, float lim) {
  const float a = fabsf(v);
  const int up = __builtin_amdgcn_frexp_mantf(a) >= lim ? 1 : 0;
  return a == 0.0f ? kNoExp : __builtin_amdgcn_frexp_expf(a) + up;
}
__device__ __forceinline__ int lane_exp(double v, double lim) {
  const double a = fabs(v);
  const int up = __builtin_amdgcn_frexp_mant(a) >= lim ? 1 : 0;
  return a == 0.0 ? kNoExp : __builtin_amdgcn_frexp_exp(a) + up;
}
// The exponent of this lane's block of B (32 or 64) lanes.
template <typename T>
__device__ __forceinline__ int block_exp(T v, int B, int w, int lane) {
  const int le = lane_exp(v, exp_lim(v, w));
  return B == 64 ? block_max_int<6>(le, lane) : block_max_int<5>(le, lane);
}

// Quantise the value v held by this lane into its block (the lanes of one
// group of B lanes form one block; every lane of the wave active).  Returns
// the code; *e_out the exponent (kZeroExp for an all-zero block).
__device__ __forceinline__ int64_t quantise_lane(double v, int B, int w, int* e_out) {
  const int E = block_exp(v, B, w, static_cast<int>(threadIdx.x & 63));
  if (E == kNoExp) {
    *e_out = kZeroExp;
    return 0;
  }
  *e_out = E;
  return static_cast<int64_t>(rint(ldexp(v, w - 1 - E)));
}

// Quantise a float32 value; identical codes to quantise_lane for w <= 24:
// a float scaled by a power of two stays exact, and results in the float
// subnormal range lie far below 1/2 and round to zero either way.
__device__ __forceinline__ int32_t quantise_lane_f32(float v, int B, int w, int lane, int* e_out) {
  const int E = block_exp(v, B, w, lane);
  if (E == kNoExp) {
    *e_out = kZeroExp;
    return 0;
  }
  *e_out = E;
  return static_cast<int32_t>(rintf(ldexpf(v, w - 1 - E)));
}

// Store the 64 codes held by the 64 lanes of a wave at values base..base+63.
// For the 12-bit container lanes 0..23 each assemble one 32-bit word;
// `limit` is the number of values that may be written (whole blocks).
__device__ __forceinline__ void store_codes_wave(const SecRef& s, int64_t base, int lane,
                                                 int64_t m, int64_t limit) {
  if (s.cbits != 12) {
    if (base + lane < limit) store_code(s, base + lane, m);
    return;
  }
  const uint32_t c = static_cast<uint32_t>(m) & 0xFFFu;
  const int bit0 = 32 * lane;
  const int v0 = bit0 / 12;
  uint64_t acc = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = v0 + j;
    const uint32_t cv = __shfl(c, v & 63, 64);
    const int sh = 12 * v - bit0;
    if (v < 64 && sh < 32) acc |= (sh >= 0) ? (static_cast<uint64_t>(cv) << sh) : (cv >> (-sh));
  }
  // words of this wave: 24; word t covers values [8t/3, ...), write only if
  // every value it covers lies below `limit` (limit is a multiple of 32)
  if (lane < 24 && base + (lane * 32 + 31) / 12 < limit)
    static_cast<uint32_t*>(s.codes)[(base / 64) * 24 + lane] = static_cast<uint32_t>(acc);
}

// ------------------------------------------------------------------ levels
struct Geom {
  int32_t dim;    // 2 or 3
  int32_t level;  // n = 2^level intervals per axis
  int32_t n;
  int64_t size;   // n^dim
};

__device__ __forceinline__ void unflatten(const Geom& g, int64_t idx, int& i, int& j, int& k) {
  i = static_cast<int>(idx & (g.n - 1));
  j = static_cast<int>((idx >> g.level) & (g.n - 1));
  k = g.dim == 3 ? static_cast<int>(idx >> (2 * g.level)) : 0;
}

__device__ __forceinline__ int64_t flat(const Geom& g, int i, int j, int k) {
  return g.dim == 3 ? ((static_cast<int64_t>(k) << (2 * g.level)) | (static_cast<int64_t>(j) << g.level) | i)
                    : ((static_cast<int64_t>(j) << g.level) | i);
}

// Value at (i, j, k); the far boundary node (index n) is an implicit 0.
template <typename T>
__device__ __forceinline__ T at(const T* u, const Geom& g, int i, int j, int k) {
  if (i >= g.n || j >= g.n || k >= g.n) return T(0);
  return u[flat(g, i, j, k)];
}

__device__ __forceinline__ bool is_interior(const Geom& g, int i, int j, int k) {
  return i > 0 && j > 0 && (g.dim == 2 || k > 0);
}

// Edge coefficients k[0..2d-1] (order -x, +x, -y, +y, -z, +z) at interior
// node (i, j, k) from the cell array `kap` (n^dim cells of this level).
template <typename T>
__device__ __forceinline__ void edge_coeffs(const T* kap, const Geom& g, int i, int j, int k, T* ke) {
  auto K3 = [&](int kc, int jc, int ic) { return kap[flat(g, ic, jc, kc)]; };
  if (g.dim == 3) {
    const T q = T(0.25);
    ke[0] = (((K3(k - 1, j - 1, i - 1) + K3(k - 1, j, i - 1)) + K3(k, j - 1, i - 1)) + K3(k, j, i - 1)) * q;
    ke[1] = (((K3(k - 1, j - 1, i) + K3(k - 1, j, i)) + K3(k, j - 1, i)) + K3(k, j, i)) * q;
    ke[2] = (((K3(k - 1, j - 1, i - 1) + K3(k - 1, j - 1, i)) + K3(k, j - 1, i - 1)) + K3(k, j - 1, i)) * q;
    ke[3] = (((K3(k - 1, j, i - 1) + K3(k - 1, j, i)) + K3(k, j, i - 1)) + K3(k, j, i)) * q;
    ke[4] = (((K3(k - 1, j - 1, i - 1) + K3(k - 1, j - 1, i)) + K3(k - 1, j, i - 1)) + K3(k - 1, j, i)) * q;
    ke[5] = (((K3(k, j - 1, i - 1) + K3(k, j - 1, i)) + K3(k, j, i - 1)) + K3(k, j, i)) * q;
  } else {
    const T q = T(0.5);
    ke[0] = (K3(0, j - 1, i - 1) + K3(0, j, i - 1)) * q;
    ke[1] = (K3(0, j - 1, i) + K3(0, j, i)) * q;
    ke[2] = (K3(0, j - 1, i - 1) + K3(0, j - 1, i)) * q;
    ke[3] = (K3(0, j, i - 1) + K3(0, j, i)) * q;
  }
}

// (A u)_p at an interior node; kap == nullptr selects Poisson.
template <typename T>
__device__ __forceinline__ T apply_A(const T* u, const T* kap, const Geom& g, int i, int j, int k, T inv_h2) {
  const T up = u[flat(g, i, j, k)];
  const T nb[6] = {at(u, g, i - 1, j, k), at(u, g, i + 1, j, k), at(u, g, i, j - 1, k),
                   at(u, g, i, j + 1, k), g.dim == 3 ? at(u, g, i, j, k - 1) : T(0),
                   g.dim == 3 ? at(u, g, i, j, k + 1) : T(0)};
  const int nd = 2 * g.dim;
  T s;
  if (kap == nullptr) {
    s = T(nd) * up;
    for (int t = 0; t < nd; ++t) s = s - nb[t];
  } else {
    T ke[6];
    edge_coeffs(kap, g, i, j, k, ke);
    s = ke[0] * (up - nb[0]);
    for (int t = 1; t < nd; ++t) s = s + ke[t] * (up - nb[t]);
  }
  return s * inv_h2;
}

// Diagonal of A at an interior node (diffusion).
template <typename T>
__device__ __forceinline__ T diag_A(const T* kap, const Geom& g, int i, int j, int k, T inv_h2) {
  T ke[6];
  edge_coeffs(kap, g, i, j, k, ke);
  T s = ke[0];
  for (int t = 1; t < 2 * g.dim; ++t) s = s + ke[t];
  return s * inv_h2;
}

// fine = P coarse (d-linear interpolation); gf is the fine level.
template <typename T>
__device__ __forceinline__ T prolong_at(const T* coarse, const Geom& gc, int i, int j, int k) {
  const int ti = i >> 1, tj = j >> 1, tk = k >> 1;
  const int pi = i & 1, pj = j & 1, pk = k & 1;
  T s = T(0);
  bool first = true;
  const int nk = (gc.dim == 3) ? 1 + pk : 1;
  for (int oz = 0; oz < nk; ++oz) {
    const double wz = (gc.dim == 3 && pk) ? 0.5 : 1.0;
    for (int oy = 0; oy <= pj; ++oy) {
      const double wy = pj ? 0.5 : 1.0;
      for (int ox = 0; ox <= pi; ++ox) {
        const double wx = pi ? 0.5 : 1.0;
        const T t = static_cast<T>(wz * wy * wx) * at(coarse, gc, ti + ox, tj + oy, tk + oz);
        s = first ? t : s + t;
        first = false;
      }
    }
  }
  return s;
}

// Smoothing coefficient c of y <- y + c (rhs - A y): `cpois` for Poisson,
// omega / diag_p for diffusion.
template <typename T>
__device__ __forceinline__ T smooth_coeff(const T* kap, const Geom& g, int i, int j, int k, T inv_h2, T cpois,
                                          T omega) {
  return kap == nullptr ? cpois : omega / diag_A(kap, g, i, j, k, inv_h2);
}

// IR residual monitor.  Kernels that form an IR residual add the squares of
// its entries to one of kMonSlots partial sums (slot = workgroup id mod
// kMonSlots, kMonStride doubles apart, so that the atomics of different
// workgroups spread over cache lines); k_monitor_check sums the slots in
// order.  After the slots: [0] the smallest sum of squares seen on this FMG
// level (-1: none yet), [1] the last sum of squares.
constexpr int kMonSlots = 64, kMonStride = 16;
constexpr int kMonMin = kMonSlots * kMonStride, kMonLast = kMonMin + 1, kMonDoubles = kMonMin + 16;
__device__ __forceinline__ void monitor_add(double* mon, double a) {
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(mon + (blockIdx.x % kMonSlots) * kMonStride, a);
}

// Exact float64 solve A y = g on a coarsest level with at most 27 interior
// nodes (one thread).  One interior node: y = g / diag.  Otherwise the
// interior matrix is assembled column by column by applying A to unit
// vectors (the same arithmetic as every other use of A), factorised as
// A = L D L^T (unit lower-triangular L, diagonal D; A is symmetric positive
// definite), and solved by forward substitution, division by D and back
// substitution, every sum taken in index order.  `e` is scratch for
// g.size values and `work` for kDenseWork values (the matrix, its factor and
// three vectors; shared memory, so that the kernel needs no private arrays);
// g, y and e use the padded level layout.
constexpr int kDenseMax = 27, kDenseWork = (2 * kDenseMax + 3) * kDenseMax;
__device__ inline void coarse_solve_dense(const double* g_in, const double* kap, const Geom& g, double ih2,
                                          double* y, double* e, double* work) {
  const int kz = g.dim == 3 ? 1 : 0;
  for (int64_t t = 0; t < g.size; ++t) y[t] = 0.0;
  if (g.n == 2) {
    const int64_t c = flat(g, 1, 1, kz);
    const double diag = kap == nullptr ? static_cast<double>(2 * g.dim) * ih2 : diag_A(kap, g, 1, 1, kz, ih2);
    y[c] = g_in[c] / diag;
    return;
  }
  const int w = g.n - 1, m = g.dim == 3 ? w * w * w : w * w;
  // interior node t in C order, x fastest
  auto ii = [&](int t) { return 1 + t % w; };
  auto jj = [&](int t) { return 1 + (t / w) % w; };
  auto kk = [&](int t) { return g.dim == 3 ? 1 + t / (w * w) : 0; };
  auto node = [&](int t) { return flat(g, ii(t), jj(t), kk(t)); };
  double* const A = work;
  double* const Lf = A + kDenseMax * kDenseMax;
  double* const d = Lf + kDenseMax * kDenseMax;
  double* const z = d + kDenseMax;
  double* const x = z + kDenseMax;
  for (int64_t t = 0; t < g.size; ++t) e[t] = 0.0;
  for (int c = 0; c < m; ++c) {
    e[node(c)] = 1.0;
    for (int r = 0; r < m; ++r) A[r * m + c] = apply_A(e, kap, g, ii(r), jj(r), kk(r), ih2);
    e[node(c)] = 0.0;
  }
  for (int j = 0; j < m; ++j) {
    double s = A[j * m + j];
    for (int k = 0; k < j; ++k) s = s - (Lf[j * m + k] * Lf[j * m + k]) * d[k];
    d[j] = s;
    for (int i = j + 1; i < m; ++i) {
      double t = A[i * m + j];
      for (int k = 0; k < j; ++k) t = t - (Lf[i * m + k] * Lf[j * m + k]) * d[k];
      Lf[i * m + j] = t / d[j];
    }
  }
  for (int i = 0; i < m; ++i) {
    double s = g_in[node(i)];
    for (int k = 0; k < i; ++k) s = s - Lf[i * m + k] * z[k];
    z[i] = s;
  }
  for (int i = m - 1; i >= 0; --i) {
    double s = z[i] / d[i];
    for (int k = i + 1; k < m; ++k) s = s - Lf[k * m + i] * x[k];
    x[i] = s;
  }
  for (int i = 0; i < m; ++i) y[node(i)] = x[i];
}

}  // namespace cmg
