// Level kernels of the compact multigrid path (gfx950, wave64).
//
// One kernel per operation on one level: BFP encode / decode / widen /
// correction, operator application, d-linear interpolation, full weighting,
// weighted-Jacobi and red-black Gauss-Seidel sweeps, right-hand-side
// injection, coefficient coarsening and the coefficient gradient.  Each
// thread owns one node of the padded level layout; BFP kernels give one
// wave to 64 consecutive values (one block of 64 or two of 32) so that the
// shared exponent is a wave-level max reduction.
#include <string>
#include <type_traits>

#include "device.h"
#include "launch.h"
#include "timing.h"

namespace cmg {

constexpr int kThreads = 256;

static inline dim3 grid_for(int64_t n) { return dim3(static_cast<unsigned>((n + kThreads - 1) / kThreads)); }

// ===================================================================== BFP
template <typename T>
__global__ void __launch_bounds__(kThreads) k_encode(const T* x, int64_t n, SecRef s, int* nonfinite, T* out,
                                                     const T* __restrict__ add, SecRef u, int correct) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (static_cast<int64_t>(blockIdx.x) * kThreads + (threadIdx.x & ~63));
  const int64_t limit = limit_of(s);
  if (base >= limit) return;  // whole wave
  const int64_t i = base + lane;
  const double v = (i < n) ? static_cast<double>(x[i]) : 0.0;
  if (nonfinite != nullptr && !isfinite(v)) atomicOr(nonfinite, 1);
  int e;
  // float input and w <= 24: the float quantiser gives the same codes
  const int64_t m = (std::is_same<T, float>::value && s.w <= 24)
                        ? quantise_lane_f32(static_cast<float>(v), s.B, s.w, lane, &e)
                        : quantise_lane(v, s.B, s.w, &e);
  store_codes_wave(s, base, lane, m, limit);
  if ((lane & (s.B - 1)) == 0 && i < limit) s.exps[blk(s, i)] = static_cast<int16_t>(e);
  // the decoded value of the new code, as k_decode gives it (plus add)
  const double dv = e == kZeroExp ? 0.0 : ldexp(static_cast<double>(m), e - (s.w - 1));
  if (out != nullptr && i < n) {
    // a float result of width <= 24 rounds once either way (see decode_value_f32)
    const T d = (std::is_same<T, float>::value && s.w <= 24)
                    ? static_cast<T>(e == kZeroExp ? 0.0f : ldexpf(static_cast<float>(m), e - (s.w - 1)))
                    : static_cast<T>(dv);
    out[i] = add != nullptr ? d + add[i] : d;
  }
  // u <- Q(dec u + dec s), as k_correct computes it (u has the blocks of s)
  if (correct) {
    const double vu = (i < limit) ? decode_value(u, i) + dv : 0.0;
    int eu;
    const int64_t mu = quantise_lane(vu, u.B, corr_width(u), &eu);
    store_codes_wave(u, base, lane, mu, limit);
    if ((lane & (u.B - 1)) == 0 && i < limit) u.exps[blk(u, i)] = static_cast<int16_t>(eu);
  }
}

// Value i of a section as float with width <= 24: the code converts exactly
// and the scaling rounds once, as the conversion of decode_value's exact
// double does (a zero block's codes are 0, so its sentinel exponent
// scales 0 to 0).
__device__ __forceinline__ float decode_value_f32(const SecRef& s, int64_t i) {
  return ldexpf(static_cast<float>(load_code(s, i)), s.exps[blk(s, i)] - (s.w - 1));
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_decode(SecRef s, int64_t n, T* __restrict__ x) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i >= n) return;
  if (std::is_same<T, float>::value && s.w <= 24) x[i] = static_cast<T>(decode_value_f32(s, i));
  else x[i] = static_cast<T>(decode_value(s, i));
}

// Append k zero bits to every code (exponents unchanged).
__global__ void __launch_bounds__(kThreads) k_widen(SecRef s, int k) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const int64_t limit = limit_of(s);
  if (s.cbits == 12) {  // one thread per pair of values (three bytes)
    if (2 * t >= limit) return;
    uint8_t* b = static_cast<uint8_t*>(s.codes) + 3 * t;
    uint32_t word = b[0] | (b[1] << 8) | (b[2] << 16);
    int32_t v0 = static_cast<int32_t>(word & 0xFFFu), v1 = static_cast<int32_t>((word >> 12) & 0xFFFu);
    v0 = (v0 ^ 0x800) - 0x800;
    v1 = (v1 ^ 0x800) - 0x800;
    v0 *= (1 << k);
    v1 *= (1 << k);
    word = (static_cast<uint32_t>(v0) & 0xFFFu) | ((static_cast<uint32_t>(v1) & 0xFFFu) << 12);
    b[0] = word & 0xFF;
    b[1] = (word >> 8) & 0xFF;
    b[2] = (word >> 16) & 0xFF;
    return;
  }
  if (t >= limit) return;
  store_code(s, t, load_code(s, t) * (static_cast<int64_t>(1) << k));
}

// Codes of a whole section set to zero with 16-byte stores (every block holds
// a multiple of 16 bytes: B >= 32 values of >= 8 bits); exponents to the
// all-zero sentinel.
__global__ void __launch_bounds__(kThreads) k_zero_section(SecRef s) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  const int64_t nb = (s.n + s.B - 1) / s.B;
  const int64_t bytes = nb * s.B * s.cbits / 8;
  if (t < bytes / 16) reinterpret_cast<uint4*>(s.codes)[t] = make_uint4(0u, 0u, 0u, 0u);
  if (t < nb) s.exps[t] = kZeroExp;
}

// Encode the interior of a full node array of level g (boundary 0).
__global__ void __launch_bounds__(kThreads) k_encode_full(const double* __restrict__ full, Geom g, SecRef s,
                                                          int* nonfinite) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (static_cast<int64_t>(blockIdx.x) * kThreads + (threadIdx.x & ~63));
  const int64_t limit = limit_of(s);
  if (base >= limit) return;
  const int64_t i = base + lane;
  double v = 0.0;
  if (i < g.size) {
    int x, y, z;
    unflatten(g, i, x, y, z);
    if (is_interior(g, x, y, z)) {
      const int64_t N = g.n + 1;
      v = full[g.dim == 3 ? (static_cast<int64_t>(z) * N + y) * N + x : static_cast<int64_t>(y) * N + x];
    }
  }
  if (nonfinite != nullptr && !isfinite(v)) atomicOr(nonfinite, 1);
  int e;
  const int64_t m = quantise_lane(v, s.B, s.w, &e);
  store_codes_wave(s, base, lane, m, limit);
  if ((lane & (s.B - 1)) == 0 && i < limit) s.exps[blk(s, i)] = static_cast<int16_t>(e);
}

// Section-wise correction u' <- round(dec u' + dec y') in float64 (Alg. 3).
__global__ void __launch_bounds__(kThreads) k_correct(SecRef u, SecRef y) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (static_cast<int64_t>(blockIdx.x) * kThreads + (threadIdx.x & ~63));
  const int64_t limit = limit_of(u);
  if (base >= limit) return;
  const int64_t i = base + lane;
  const double v = (i < limit) ? decode_value(u, i) + decode_value(y, i) : 0.0;
  int e;
  const int64_t m = quantise_lane(v, u.B, corr_width(u), &e);
  store_codes_wave(u, base, lane, m, limit);
  if ((lane & (u.B - 1)) == 0 && i < limit) u.exps[blk(u, i)] = static_cast<int16_t>(e);
}

// ============================================================ level kernels
// Diffusion operator at interior node (i, j, k): (A u)_p and, when diag is
// not null, the diagonal of A.  The same arithmetic as apply_A and diag_A
// (edge coefficients as in edge_coeffs, same order), but each of the 2^d
// cells around the node is loaded once, at a fixed offset from the first.
template <typename T>
__device__ __forceinline__ void cell_edges(const T* __restrict__ kap, const Geom& g, int i, int j, int k, T* ke) {
  const int64_t n = g.n;
  if (g.dim == 3) {
    const int64_t b = flat(g, i - 1, j - 1, k - 1), n2 = n * n;
    const T c000 = kap[b], c100 = kap[b + 1], c010 = kap[b + n], c110 = kap[b + n + 1];
    const T c001 = kap[b + n2], c101 = kap[b + n2 + 1], c011 = kap[b + n2 + n], c111 = kap[b + n2 + n + 1];
    const T q = T(0.25);
    ke[0] = (((c000 + c010) + c001) + c011) * q;
    ke[1] = (((c100 + c110) + c101) + c111) * q;
    ke[2] = (((c000 + c100) + c001) + c101) * q;
    ke[3] = (((c010 + c110) + c011) + c111) * q;
    ke[4] = (((c000 + c100) + c010) + c110) * q;
    ke[5] = (((c001 + c101) + c011) + c111) * q;
  } else {
    const int64_t b = flat(g, i - 1, j - 1, 0);
    const T c00 = kap[b], c10 = kap[b + 1], c01 = kap[b + n], c11 = kap[b + n + 1];
    const T q = T(0.5);
    ke[0] = (c00 + c01) * q;
    ke[1] = (c10 + c11) * q;
    ke[2] = (c00 + c10) * q;
    ke[3] = (c01 + c11) * q;
  }
}

// Diagonal of the diffusion operator at an interior node (as diag_A).
template <typename T>
__device__ __forceinline__ T diffusion_diag(const T* __restrict__ kap, const Geom& g, int i, int j, int k,
                                            T inv_h2) {
  T ke[6];
  cell_edges(kap, g, i, j, k, ke);
  T d = ke[0];
  for (int t = 1; t < 2 * g.dim; ++t) d = d + ke[t];
  return d * inv_h2;
}

template <typename T>
__device__ __forceinline__ T diffusion_at(const T* __restrict__ u, const T* __restrict__ kap, const Geom& g, int i,
                                          int j, int k, T inv_h2, T* diag) {
  const int64_t n = g.n;
  const int64_t p = flat(g, i, j, k);
  const T up = u[p];
  T ke[6], nb[6];
  cell_edges(kap, g, i, j, k, ke);
  if (g.dim == 3) {
    const int64_t n2 = n * n;
    nb[0] = u[p - 1];
    nb[1] = i + 1 < g.n ? u[p + 1] : T(0);
    nb[2] = u[p - n];
    nb[3] = j + 1 < g.n ? u[p + n] : T(0);
    nb[4] = u[p - n2];
    nb[5] = k + 1 < g.n ? u[p + n2] : T(0);
  } else {
    nb[0] = u[p - 1];
    nb[1] = i + 1 < g.n ? u[p + 1] : T(0);
    nb[2] = u[p - n];
    nb[3] = j + 1 < g.n ? u[p + n] : T(0);
  }
  const int nd = 2 * g.dim;
  T s = ke[0] * (up - nb[0]);
  for (int t = 1; t < nd; ++t) s = s + ke[t] * (up - nb[t]);
  if (diag != nullptr) {
    T d = ke[0];
    for (int t = 1; t < nd; ++t) d = d + ke[t];
    *diag = d * inv_h2;
  }
  return s * inv_h2;
}

// out = rhs - A u on interior nodes, 0 on the boundary.
// DIFF: the diffusion operator (kap holds the cell coefficients), else
// Poisson (kap is null); one instantiation each, so neither carries the
// other's code.
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_rhs_minus_A(const T* __restrict__ rhs, const T* __restrict__ u,
                                                          const T* __restrict__ kap, Geom g, T inv_h2,
                                                          T* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= g.size) return;
  int i, j, k;
  unflatten(g, idx, i, j, k);
  if (!is_interior(g, i, j, k)) {
    out[idx] = T(0);
    return;
  }
  const T au = DIFF ? diffusion_at<T>(u, kap, g, i, j, k, inv_h2, nullptr) : apply_A<T>(u, nullptr, g, i, j, k, inv_h2);
  out[idx] = rhs[idx] - au;
}

// out = dec(gs) - A u on interior nodes, 0 on the boundary: k_decode of the
// right-hand side section followed by k_rhs_minus_A, in one pass.
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_dec_minus_A(SecRef gs, const T* __restrict__ u,
                                                          const T* __restrict__ kap, Geom g, T inv_h2,
                                                          T* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= g.size) return;
  int i, j, k;
  unflatten(g, idx, i, j, k);
  if (!is_interior(g, i, j, k)) {
    out[idx] = T(0);
    return;
  }
  const T au = DIFF ? diffusion_at<T>(u, kap, g, i, j, k, inv_h2, nullptr) : apply_A<T>(u, nullptr, g, i, j, k, inv_h2);
  out[idx] = static_cast<T>(decode_value(gs, idx)) - au;
}

// The float64 residual of iterative refinement encoded into s: t = f - A u
// on interior nodes (0 elsewhere), quantised into its blocks.  The same
// values as k_rhs_minus_A<double> followed by k_encode<double>, without the
// t array; one wave per 64 consecutive values.
template <bool DIFF>
__global__ void __launch_bounds__(kThreads) k_res_encode(const double* __restrict__ f, const double* __restrict__ u,
                                                         const double* __restrict__ kap, Geom g, double inv_h2,
                                                         SecRef s, int* nonfinite, double* mon) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (static_cast<int64_t>(blockIdx.x) * kThreads + (threadIdx.x & ~63));
  const int64_t limit = limit_of(s);
  if (base >= limit) return;  // whole wave
  const int64_t i = base + lane;
  double v = 0.0;
  if (i < g.size) {
    int x, y, z;
    unflatten(g, i, x, y, z);
    if (is_interior(g, x, y, z)) {
      const double au = DIFF ? diffusion_at<double>(u, kap, g, x, y, z, inv_h2, nullptr)
                             : apply_A<double>(u, nullptr, g, x, y, z, inv_h2);
      v = f[i] - au;
    }
  }
  if (nonfinite != nullptr && !isfinite(v)) atomicOr(nonfinite, 1);
  if (mon != nullptr) monitor_add(mon, v * v);
  int e;
  const int64_t m = quantise_lane(v, s.B, s.w, &e);
  store_codes_wave(s, base, lane, m, limit);
  if ((lane & (s.B - 1)) == 0 && i < limit) s.exps[blk(s, i)] = static_cast<int16_t>(e);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_prolong(const T* __restrict__ coarse, Geom gf, Geom gc,
                                                      T* __restrict__ fine) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gf.size) return;
  int i, j, k;
  unflatten(gf, idx, i, j, k);
  fine[idx] = prolong_at(coarse, gc, i, j, k);
}

// k_prolong on a 3-D level of at most 2^30 nodes: prolong_at's terms and
// order (z, y, x; a product by the weight, then the sum), with 32-bit
// indices; every coarse neighbour is loaded (clamped into the level) and
// the terms are chosen by selects, so that no load sits under a branch.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_prolong3(const T* __restrict__ coarse, int lf, T* __restrict__ fine) {
  const uint32_t idx = blockIdx.x * kThreads + threadIdx.x;
  const int nf = 1 << lf, lc = lf - 1, nc = nf >> 1;
  if (idx >= (1u << (3 * lf))) return;
  const int i = idx & (nf - 1), j = (idx >> lf) & (nf - 1), k = idx >> (2 * lf);
  const int ti = i >> 1, tj = j >> 1, tk = k >> 1;
  const bool px = i & 1, py = j & 1, pz = k & 1;
  const T w = static_cast<T>((px ? 0.5 : 1.0) * (py ? 0.5 : 1.0) * (pz ? 0.5 : 1.0));
  // coarse value at (ti + ox, tj + oy, tk + oz); the far boundary node nc is 0
  auto at = [&](int ox, int oy, int oz) {
    const int a = ti + ox, b = tj + oy, c = tk + oz;
    const uint32_t q = (static_cast<uint32_t>(min(c, nc - 1)) << (2 * lc)) |
                       (static_cast<uint32_t>(min(b, nc - 1)) << lc) | static_cast<uint32_t>(min(a, nc - 1));
    const T v = coarse[q];
    return (a < nc && b < nc && c < nc) ? v : T(0);
  };
  T s = w * at(0, 0, 0);
  T t = s + w * at(1, 0, 0);
  s = px ? t : s;
  t = s + w * at(0, 1, 0);
  s = py ? t : s;
  t = s + w * at(1, 1, 0);
  s = (px && py) ? t : s;
  t = s + w * at(0, 0, 1);
  s = pz ? t : s;
  t = s + w * at(1, 0, 1);
  s = (pz && px) ? t : s;
  t = s + w * at(0, 1, 1);
  s = (pz && py) ? t : s;
  t = s + w * at(1, 1, 1);
  s = (pz && px && py) ? t : s;
  fine[idx] = s;
}

// out = dec(section) + P coarse, float64 (one step of the decode chain).
__global__ void __launch_bounds__(kThreads) k_prolong_add_dec(SecRef sec, const double* __restrict__ coarse,
                                                              Geom gf, Geom gc, double* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gf.size) return;
  int i, j, k;
  unflatten(gf, idx, i, j, k);
  out[idx] = decode_value(sec, idx) + prolong_at(coarse, gc, i, j, k);
}

// (R fine) at coarse node (I, J, K) (full weighting; 0 off the interior).
template <typename T>
__device__ __forceinline__ T restrict_at(const T* __restrict__ fine, const Geom& gc, const Geom& gf, int I, int J,
                                         int K) {
  if (!is_interior(gc, I, J, K)) return T(0);
  T s = T(0);
  bool first = true;
  const int z0 = gc.dim == 3 ? -1 : 0, z1 = gc.dim == 3 ? 1 : 0;
  for (int oz = z0; oz <= z1; ++oz) {
    const double wz = gc.dim == 3 ? (oz == 0 ? 0.5 : 0.25) : 1.0;
    for (int oy = -1; oy <= 1; ++oy) {
      const double wy = oy == 0 ? 0.5 : 0.25;
      for (int ox = -1; ox <= 1; ++ox) {
        const double wx = ox == 0 ? 0.5 : 0.25;
        const int kf = gc.dim == 3 ? 2 * K + oz : 0;
        const T t = static_cast<T>(wz * wy * wx) * fine[flat(gf, 2 * I + ox, 2 * J + oy, kf)];
        s = first ? t : s + t;
        first = false;
      }
    }
  }
  return s;
}

// coarse = R fine (full weighting); gc is the coarse level.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_restrict(const T* __restrict__ fine, Geom gc, Geom gf,
                                                       T* __restrict__ coarse) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gc.size) return;
  int I, J, K;
  unflatten(gc, idx, I, J, K);
  coarse[idx] = restrict_at(fine, gc, gf, I, J, K);
}

// s = Q(R fine): k_restrict followed by k_encode, without the coarse array
// (one wave per 64 consecutive coarse values).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_restrict_encode(const T* __restrict__ fine, Geom gc, Geom gf, SecRef s,
                                                              int* nonfinite) {
  const int lane = threadIdx.x & 63;
  const int64_t base = (static_cast<int64_t>(blockIdx.x) * kThreads + (threadIdx.x & ~63));
  const int64_t limit = limit_of(s);
  if (base >= limit) return;  // whole wave
  const int64_t i = base + lane;
  double v = 0.0;
  if (i < gc.size) {
    int I, J, K;
    unflatten(gc, i, I, J, K);
    v = static_cast<double>(restrict_at(fine, gc, gf, I, J, K));
  }
  if (nonfinite != nullptr && !isfinite(v)) atomicOr(nonfinite, 1);
  int e;
  const int64_t m = (std::is_same<T, float>::value && s.w <= 24)
                        ? quantise_lane_f32(static_cast<float>(v), s.B, s.w, lane, &e)
                        : quantise_lane(v, s.B, s.w, &e);
  store_codes_wave(s, base, lane, m, limit);
  if ((lane & (s.B - 1)) == 0 && i < limit) s.exps[blk(s, i)] = static_cast<int16_t>(e);
}

template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_jacobi(const T* __restrict__ y, const T* __restrict__ rhs,
                                                     const T* __restrict__ kap, Geom g, T inv_h2, T cpois,
                                                     T omega, T* __restrict__ ynew) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= g.size) return;
  int i, j, k;
  unflatten(g, idx, i, j, k);
  if (!is_interior(g, i, j, k)) {
    ynew[idx] = T(0);
    return;
  }
  if (DIFF) {
    T d;
    const T r = rhs[idx] - diffusion_at<T>(y, kap, g, i, j, k, inv_h2, &d);
    const T c = omega / d;
    ynew[idx] = y[idx] + c * r;
  } else {
    const T r = rhs[idx] - apply_A<T>(y, nullptr, g, i, j, k, inv_h2);
    ynew[idx] = y[idx] + cpois * r;
  }
}

// One thread per node of the colour: thread t takes node i = 2 (t mod n/2)
// + ((j + k + colour) & 1) of row t div (n/2), so every lane of a wave has
// a node to update (n is even on every level).
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_rbgs(T* __restrict__ y, const T* __restrict__ rhs,
                                                   const T* __restrict__ kap, Geom g, T inv_h2, T cpois,
                                                   int colour) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (t >= (g.size >> 1)) return;
  const int64_t row = t >> (g.level - 1);  // j + n k
  const int j = static_cast<int>(row & (g.n - 1));
  const int k = g.dim == 3 ? static_cast<int>(row >> g.level) : 0;
  const int i = 2 * static_cast<int>(t & ((g.n >> 1) - 1)) + ((j + k + colour) & 1);
  if (!is_interior(g, i, j, k)) return;
  const int64_t idx = flat(g, i, j, k);
  if (DIFF) {
    T d;
    const T r = rhs[idx] - diffusion_at<T>(y, kap, g, i, j, k, inv_h2, &d);
    const T c = T(1) / d;
    y[idx] = y[idx] + c * r;
  } else {
    const T r = rhs[idx] - apply_A<T>(y, nullptr, g, i, j, k, inv_h2);
    y[idx] = y[idx] + cpois * r;
  }
}

// The first red half-sweep from y = 0, over all nodes: red interior nodes
// take 0 + c (rhs - A 0) = 0 + c rhs (A 0 is +0, so this is what k_rbgs
// computes after a fill with zeros), every other node 0.
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_rbgs_zero(T* __restrict__ y, const T* __restrict__ rhs,
                                                        const T* __restrict__ kap, Geom g, T inv_h2, T cpois) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= g.size) return;
  int i, j, k;
  unflatten(g, idx, i, j, k);
  if (!is_interior(g, i, j, k) || ((i + j + k) & 1) != 0) {
    y[idx] = T(0);
    return;
  }
  const T c = DIFF ? T(1) / diffusion_diag<T>(kap, g, i, j, k, inv_h2) : cpois;
  y[idx] = T(0) + c * (rhs[idx] - T(0));
}

// A full red-black Gauss-Seidel sweep of a 3-D level (n >= 64) in one
// launch, out of place (yin -> yout, so that no workgroup reads a value
// another one has already replaced).  A workgroup owns a 64 x kSwTY tile
// and marches along z through a chunk of TZ planes: at step p it updates
// the red nodes of plane p on the tile and a one-node halo, then the black
// nodes of plane p - 1 on the tile, whose red neighbours (planes p - 2 to
// p) are updated by then, and writes plane p - 1.  Planes of y pass through
// a ring of four LDS planes holding the tile and a two-node halo.  Every
// node gets the arithmetic of k_rbgs (same operands in the same order), so
// the sweep equals a red and a black half-sweep launch bit for bit.  With
// ZERO, y is taken as 0 (the first sweep from zero) and yin is not read;
// with SEC, y is the decoded section ysec (as k_decode gives it) and yin is
// not read.
constexpr int kSwTX = 64, kSwTY = 8, kSwNT = 256;
template <typename T, bool DIFF, bool ZERO, bool SEC>
__global__ void __launch_bounds__(kSwNT) k_rbgs_sweep(const T* __restrict__ yin, SecRef ysec, T* __restrict__ yout,
                                                      const T* __restrict__ rhs, const T* __restrict__ kap, Geom g,
                                                      T inv_h2, T cpois, int TZ) {
  constexpr int W = kSwTX + 4, H = kSwTY + 4, PL = W * H;
  __shared__ T ring[4 * PL];
  const int tid = threadIdx.x;
  const int n = g.n;
  const int ntx = n / kSwTX, nty = n / kSwTY;
  const int bx = blockIdx.x % ntx, by = (blockIdx.x / ntx) % nty, bz = blockIdx.x / (ntx * nty);
  const int X0 = bx * kSwTX, Y0 = by * kSwTY, Z0 = bz * TZ;
  const int64_t pn = static_cast<int64_t>(n) * n;  // values per plane
  auto slot = [&](int q) { return ring + (q & 3) * PL; };
  // plane q of y on the tile and a two-node halo; 0 outside the level
  auto load = [&](int q) {
    T* d = slot(q);
    for (int t = tid; t < PL; t += kSwNT) {
      const int ly = t / W, lx = t - ly * W;
      const int gx = X0 - 2 + lx, gy = Y0 - 2 + ly;
      T v = T(0);
      if (!ZERO && q >= 0 && q < n && gx >= 0 && gx < n && gy >= 0 && gy < n) {
        const int64_t idx = q * pn + static_cast<int64_t>(gy) * n + gx;
        v = SEC ? static_cast<T>(decode_value(ysec, idx)) : yin[idx];
      }
      d[t] = v;
    }
  };
  // new value of interior node (lx, ly) of plane q (neighbours in the ring)
  auto update = [&](int lx, int ly, int q) -> T {
    const T* c = slot(q);
    const int t = ly * W + lx;
    const int gx = X0 - 2 + lx, gy = Y0 - 2 + ly;
    const T up = c[t];
    const T nb[6] = {c[t - 1], c[t + 1], c[t - W], c[t + W], slot(q - 1)[t], slot(q + 1)[t]};
    T s, cc;
    if (DIFF) {
      T ke[6];
      cell_edges(kap, g, gx, gy, q, ke);
      s = ke[0] * (up - nb[0]);
      for (int e = 1; e < 6; ++e) s = s + ke[e] * (up - nb[e]);
      T d = ke[0];
      for (int e = 1; e < 6; ++e) d = d + ke[e];
      cc = T(1) / (d * inv_h2);
    } else {
      s = T(6) * up;
      for (int e = 0; e < 6; ++e) s = s - nb[e];
      cc = cpois;
    }
    const T r = rhs[q * pn + static_cast<int64_t>(gy) * n + gx] - s * inv_h2;
    return up + cc * r;
  };
  load(Z0 - 2);
  load(Z0 - 1);
  for (int p = Z0 - 1; p <= Z0 + TZ; ++p) {
    load(p + 1);
    __syncthreads();
    // Red nodes of plane p on the tile and its one-node halo (they read only
    // black neighbours).  X0 is even, so in row ly the red nodes are every
    // other lx from lx0 = 2 - ((gy + p) & 1): 33 per row.
    if (p >= 1 && p < n) {
      T* c = slot(p);
      constexpr int RW = (W - 2) / 2;
      for (int t = tid; t < RW * (H - 2); t += kSwNT) {
        const int ly = 1 + t / RW, gy = Y0 - 2 + ly;
        const int lx = 2 - ((gy + p) & 1) + 2 * (t % RW), gx = X0 - 2 + lx;
        if (gx >= 1 && gx < n && gy >= 1 && gy < n) c[ly * W + lx] = update(lx, ly, p);
      }
    }
    __syncthreads();
    // Black nodes of plane q = p - 1 on the tile, and plane q out: a
    // thread takes the pair of nodes at lx and lx + 1 (lx even) of a row, one
    // red and one black.
    const int q = p - 1;
    if (q >= Z0 && q < Z0 + TZ) {
      const T* c = slot(q);
      static_assert(kSwTX * kSwTY % (2 * kSwNT) == 0, "whole pairs per thread");
      for (int t = tid; t < kSwTX * kSwTY / 2; t += kSwNT) {
        const int ly = 2 + t / (kSwTX / 2), gy = Y0 + ly - 2;
        const int lx = 2 + 2 * (t % (kSwTX / 2)), gx = X0 + lx - 2;
        const int lb = lx + ((gx + gy + q + 1) & 1);  // the black node of the pair
        const int gb = X0 + lb - 2;
        T v[2] = {c[ly * W + lx], c[ly * W + lx + 1]};
        if (q >= 1 && gb >= 1 && gy >= 1) v[lb - lx] = update(lb, ly, q);
        T* o = yout + q * pn + static_cast<int64_t>(gy) * n + gx;
        o[0] = v[0];
        o[1] = v[1];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------ plain FP64 multigrid
// The plain path keeps u, r and y per level and no further level arrays;
// these kernels fuse what it would otherwise stage through one.

// out = (T)(f - A u) on interior nodes (0 elsewhere), float64 arithmetic:
// f is sampled from the finest node array (injection), u is the padded
// float64 solution of level g.  The same values as k_inject, k_rhs_minus_A
// <double> and k_convert<double, T>; the squares of the float64 residual
// go to the monitor slots, non-finite values to nonfinite.
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_residual_full(const double* __restrict__ f, int Lfull,
                                                            const double* __restrict__ u,
                                                            const double* __restrict__ kap, Geom g, double inv_h2,
                                                            T* __restrict__ out, int* nonfinite, double* mon) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  double t = 0.0;
  if (idx < g.size) {
    int i, j, k;
    unflatten(g, idx, i, j, k);
    if (is_interior(g, i, j, k)) {
      const int64_t N = (int64_t{1} << Lfull) + 1, st = int64_t{1} << (Lfull - g.level);
      const int64_t fi = g.dim == 3 ? ((k * st) * N + j * st) * N + i * st : (j * st) * N + i * st;
      const double au = DIFF ? diffusion_at<double>(u, kap, g, i, j, k, inv_h2, nullptr)
                             : apply_A<double>(u, nullptr, g, i, j, k, inv_h2);
      t = f[fi] - au;
    }
    out[idx] = static_cast<T>(t);
    if (!isfinite(t)) atomicOr(nonfinite, 1);
  }
  monitor_add(mon, t * t);
}

// rc = R (r - A y) (full weighting of the residual, formed on the fly at
// the 3^d fine nodes of each coarse node): the same values as
// k_rhs_minus_A<T> followed by k_restrict<T>.
template <typename T, bool DIFF>
__global__ void __launch_bounds__(kThreads) k_restrict_residual(const T* __restrict__ r, const T* __restrict__ y,
                                                                const T* __restrict__ kap, Geom gc, Geom gf,
                                                                T inv_h2, T* __restrict__ rc) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gc.size) return;
  int I, J, K;
  unflatten(gc, idx, I, J, K);
  if (!is_interior(gc, I, J, K)) {
    rc[idx] = T(0);
    return;
  }
  T s = T(0);
  bool first = true;
  const int z0 = gc.dim == 3 ? -1 : 0, z1 = gc.dim == 3 ? 1 : 0;
  for (int oz = z0; oz <= z1; ++oz) {
    const double wz = gc.dim == 3 ? (oz == 0 ? 0.5 : 0.25) : 1.0;
    for (int oy = -1; oy <= 1; ++oy) {
      const double wy = oy == 0 ? 0.5 : 0.25;
      for (int ox = -1; ox <= 1; ++ox) {
        const double wx = ox == 0 ? 0.5 : 0.25;
        const int fi = 2 * I + ox, fj = 2 * J + oy, fk = gc.dim == 3 ? 2 * K + oz : 0;
        const T au = DIFF ? diffusion_at<T>(y, kap, gf, fi, fj, fk, inv_h2, nullptr)
                          : apply_A<T>(y, nullptr, gf, fi, fj, fk, inv_h2);
        const T res = r[flat(gf, fi, fj, fk)] - au;  // every fine node here is interior
        const T t = static_cast<T>(wz * wy * wx) * res;
        s = first ? t : s + t;
        first = false;
      }
    }
  }
  rc[idx] = s;
}

// y = y + P yc in place (k_prolong and k_add in one pass).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_prolong_add(const T* __restrict__ coarse, Geom gf, Geom gc,
                                                          T* __restrict__ y) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gf.size) return;
  int i, j, k;
  unflatten(gf, idx, i, j, k);
  y[idx] = y[idx] + prolong_at(coarse, gc, i, j, k);
}

// u = u + (double) y (k_convert<T, double> and k_add<double> in one pass).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_add_correction(double* __restrict__ u, const T* __restrict__ y,
                                                             int64_t n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < n) u[idx] = u[idx] + static_cast<double>(y[idx]);
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_add(const T* __restrict__ a, const T* __restrict__ b,
                                                  T* __restrict__ out, int64_t n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < n) out[idx] = a[idx] + b[idx];
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fill(T* __restrict__ x, T v, int64_t n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < n) x[idx] = v;
}

template <typename S, typename D>
__global__ void __launch_bounds__(kThreads) k_convert(const S* __restrict__ a, D* __restrict__ b, int64_t n) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < n) b[idx] = static_cast<D>(a[idx]);
}

// Padded level array <- full node array of level L sampled with stride
// 2^(L - level); boundary set to 0.
__global__ void __launch_bounds__(kThreads) k_inject(const double* __restrict__ full, int L, Geom g,
                                                     double* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= g.size) return;
  int i, j, k;
  unflatten(g, idx, i, j, k);
  if (!is_interior(g, i, j, k)) {
    out[idx] = 0.0;
    return;
  }
  const int64_t N = (static_cast<int64_t>(1) << L) + 1;
  const int s = 1 << (L - g.level);
  const int64_t src = g.dim == 3 ? ((static_cast<int64_t>(k) * s * N + static_cast<int64_t>(j) * s) * N + i * s)
                                 : (static_cast<int64_t>(j) * s * N + i * s);
  out[idx] = full[src];
}

// Full node array ((n+1)^dim) <- padded level array; far boundary 0.
__global__ void __launch_bounds__(kThreads) k_to_full(const double* __restrict__ pad, Geom g,
                                                      double* __restrict__ full) {
  const int64_t N = g.n + 1;
  const int64_t total = g.dim == 3 ? N * N * N : N * N;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= total) return;
  const int i = static_cast<int>(idx % N);
  const int j = static_cast<int>((idx / N) % N);
  const int k = g.dim == 3 ? static_cast<int>(idx / (N * N)) : 0;
  full[idx] = (i < g.n && j < g.n && k < g.n) ? pad[flat(g, i, j, k)] : 0.0;
}

// Exact float64 solve on the coarsest level (one interior node, or up to 27
// by a dense L D L^T factorisation), one thread.
__global__ void k_coarse_single(const double* __restrict__ gin, const double* __restrict__ kap, Geom g,
                                double inv_h2, double* __restrict__ y) {
  __shared__ double e[64];
  __shared__ double work[kDenseWork];
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  coarse_solve_dense(gin, kap, g, inv_h2, y, e, work);
}

// ================================================================ kappa
// Coarse cell = mean of its 2^d children (C order), float64.
__global__ void __launch_bounds__(kThreads) k_coarsen_kappa(const double* __restrict__ fine, Geom gc, Geom gf,
                                                            double* __restrict__ coarse) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gc.size) return;
  int I, J, K;
  unflatten(gc, idx, I, J, K);
  double s = 0.0;
  bool first = true;
  const int nz = gc.dim == 3 ? 2 : 1;
  for (int oz = 0; oz < nz; ++oz)
    for (int oy = 0; oy < 2; ++oy)
      for (int ox = 0; ox < 2; ++ox) {
        const double t = fine[flat(gf, 2 * I + ox, 2 * J + oy, gc.dim == 3 ? 2 * K + oz : 0)];
        s = first ? t : s + t;
        first = false;
      }
  coarse[idx] = s * (gc.dim == 3 ? 0.125 : 0.25);
}

// flags[0] |= 1 if any value <= 0, flags[1] |= 1 if any value is not finite.
__global__ void __launch_bounds__(kThreads) k_check_positive(const double* __restrict__ x, int64_t n, int* flags) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= n) return;
  const double v = x[idx];
  if (!isfinite(v)) atomicOr(flags + 1, 1);
  else if (!(v > 0.0)) atomicOr(flags, 1);
}

__global__ void __launch_bounds__(kThreads) k_check_finite(const double* __restrict__ x, int64_t n, int* flags) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < n && !isfinite(x[idx])) atomicOr(flags + 1, 1);
}

// dJ/dkappa per cell from full node arrays u, lambda ((n+1)^dim).
__global__ void __launch_bounds__(kThreads) k_grad_kappa(const double* __restrict__ u, const double* __restrict__ lam,
                                                         Geom gcell, int accumulate, double* __restrict__ grad) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= gcell.size) return;
  int ic, jc, kc;
  unflatten(gcell, idx, ic, jc, kc);
  const int64_t N = gcell.n + 1;
  auto node = [&](int k, int j, int i) { return (static_cast<int64_t>(k) * N + j) * N + i; };
  double s = 0.0;
  bool first = true;
  auto add = [&](int64_t lo, int64_t hi) {
    const double t = (lam[hi] - lam[lo]) * (u[hi] - u[lo]);
    s = first ? t : s + t;
    first = false;
  };
  if (gcell.dim == 3) {
    for (int oz = 0; oz < 2; ++oz)  // edges along x
      for (int oy = 0; oy < 2; ++oy) add(node(kc + oz, jc + oy, ic), node(kc + oz, jc + oy, ic + 1));
    for (int oz = 0; oz < 2; ++oz)  // edges along y
      for (int ox = 0; ox < 2; ++ox) add(node(kc + oz, jc, ic + ox), node(kc + oz, jc + 1, ic + ox));
    for (int oy = 0; oy < 2; ++oy)  // edges along z
      for (int ox = 0; ox < 2; ++ox) add(node(kc, jc + oy, ic + ox), node(kc + 1, jc + oy, ic + ox));
  } else {
    for (int oy = 0; oy < 2; ++oy) add(node(0, jc + oy, ic), node(0, jc + oy, ic + 1));
    for (int ox = 0; ox < 2; ++ox) add(node(0, jc, ic + ox), node(0, jc + 1, ic + ox));
  }
  const double fac = -(static_cast<double>(gcell.n) * static_cast<double>(gcell.n)) * (gcell.dim == 3 ? 0.25 : 0.5);
  const double v = s * fac;
  grad[idx] = accumulate ? grad[idx] + v : v;
}

// out[0] += sum x^2 (for residual-norm statistics; summation order is
// unspecified).
__global__ void __launch_bounds__(kThreads) k_sumsq(const double* __restrict__ x, int64_t n, double* mon) {
  double a = 0.0;
  for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; idx < n;
       idx += static_cast<int64_t>(gridDim.x) * kThreads)
    a += x[idx] * x[idx];
  monitor_add(mon, a);
}

// Clears the monitor's partial sums (and, on entering an FMG level, its
// smallest sum of squares).
__global__ void k_monitor_reset(double* mon, int entry) {
  for (int t = threadIdx.x; t < kMonSlots; t += blockDim.x) mon[t * kMonStride] = 0.0;
  if (entry && threadIdx.x == 0) mon[kMonMin] = -1.0;
}

// Sum of squares of this IR residual from the slots; a residual norm above
// `growth` times the smallest one of the FMG level so far marks the solve
// as not converging (flags[2] = level).
__global__ void k_monitor_check(double* mon, int* flags, int level, double growth) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int t = 0; t < kMonSlots; ++t) s += mon[t * kMonStride];
  const double lo = mon[kMonMin];
  if (lo >= 0.0 && s > growth * growth * lo) atomicMax(flags + 2, level);
  if (lo < 0.0 || s < lo) mon[kMonMin] = s;
  mon[kMonLast] = s;
}

// ============================================================== launchers
thread_local KernelTiming* g_timing = nullptr;

template <typename T> struct TName;
template <> struct TName<float> { static constexpr const char* s = "float"; };
template <> struct TName<double> { static constexpr const char* s = "double"; };

// Launch `kernel` over n threads, timed when a timing sink is active.
#define CMG_TLAUNCH(name, nbytes, kernel, n, stream, ...)                                 \
  do {                                                                                    \
    if (g_timing != nullptr) g_timing->begin((name), static_cast<double>(nbytes), stream); \
    hipLaunchKernelGGL(kernel, grid_for(n), dim3(kThreads), 0, stream, __VA_ARGS__);       \
    if (g_timing != nullptr) g_timing->end(stream);                                       \
  } while (0)

static inline std::string tname(const char* base, const char* t) { return std::string(base) + "<" + t + ">"; }
static inline double sec_bytes(const SecRef& s) {
  const double nb = static_cast<double>((s.n + s.B - 1) / s.B);
  return nb * s.B * s.cbits / 8.0 + 2.0 * nb;
}

template <typename T>
void launch_encode(const T* x, int64_t n, const SecRef& s, int* nonfinite, hipStream_t st) {
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  CMG_TLAUNCH(tname("k_encode", TName<T>::s).c_str(), n * sizeof(T) + sec_bytes(s), k_encode<T>, limit, st, x, n,
              s, nonfinite, static_cast<T*>(nullptr), static_cast<const T*>(nullptr), s, 0);
}
template <typename T>
void launch_encode_dec(const T* x, int64_t n, const SecRef& s, int* nonfinite, T* out, const T* add,
                       const SecRef* correct_u, hipStream_t st) {
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  const double b = n * sizeof(T) * (out != nullptr ? (add != nullptr ? 3.0 : 2.0) : 1.0) + sec_bytes(s) +
                   (correct_u != nullptr ? 2.0 * sec_bytes(*correct_u) : 0.0);
  CMG_TLAUNCH(tname("k_encode", TName<T>::s).c_str(), b, k_encode<T>, limit, st, x, n, s, nonfinite, out, add,
              correct_u != nullptr ? *correct_u : s, correct_u != nullptr ? 1 : 0);
}
template <typename T>
void launch_decode(const SecRef& s, int64_t n, T* x, hipStream_t st) {
  CMG_TLAUNCH(tname("k_decode", TName<T>::s).c_str(), n * sizeof(T) + sec_bytes(s), k_decode<T>, n, st, s, n, x);
}
void launch_encode_full(const double* full, int L, const Geom& g, const SecRef& s, int* nonfinite, hipStream_t st) {
  (void)L;
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  CMG_TLAUNCH("k_encode_full", 8.0 * g.size + sec_bytes(s), k_encode_full, limit, st, full, g, s, nonfinite);
}
void launch_widen(const SecRef& s, int k, hipStream_t st) {
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  CMG_TLAUNCH("k_widen", 2.0 * (sec_bytes(s) - 2.0 * (limit / s.B)), k_widen, s.cbits == 12 ? limit / 2 : limit,
              st, s, k);
}
void launch_zero_section(const SecRef& s, hipStream_t st) {
  const int64_t nb = (s.n + s.B - 1) / s.B;
  const int64_t quads = nb * s.B * s.cbits / 8 / 16;
  CMG_TLAUNCH("k_zero_section", sec_bytes(s), k_zero_section, quads > nb ? quads : nb, st, s);
}
void launch_correct(const SecRef& u, const SecRef& y, hipStream_t st) {
  const int64_t limit = ((u.n + u.B - 1) / u.B) * u.B;
  CMG_TLAUNCH("k_correct", 2.0 * sec_bytes(u) + sec_bytes(y), k_correct, limit, st, u, y);
}
template <typename T>
void launch_rhs_minus_A(const T* rhs, const T* u, const T* kap, const Geom& g, T inv_h2, T* out, hipStream_t st) {
  const double b = (3.0 + (kap ? 1.0 : 0.0)) * g.size * sizeof(T);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_rhs_minus_A", TName<T>::s).c_str(), b, (k_rhs_minus_A<T, true>), g.size, st, rhs, u, kap, g,
                inv_h2, out);
  else
    CMG_TLAUNCH(tname("k_rhs_minus_A", TName<T>::s).c_str(), b, (k_rhs_minus_A<T, false>), g.size, st, rhs, u, kap,
                g, inv_h2, out);
}
template <typename T>
void launch_dec_minus_A(const SecRef& gs, const T* u, const T* kap, const Geom& g, T inv_h2, T* out, hipStream_t st) {
  const double b = (2.0 + (kap ? 1.0 : 0.0)) * g.size * sizeof(T) + sec_bytes(gs);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_dec_minus_A", TName<T>::s).c_str(), b, (k_dec_minus_A<T, true>), g.size, st, gs, u, kap, g,
                inv_h2, out);
  else
    CMG_TLAUNCH(tname("k_dec_minus_A", TName<T>::s).c_str(), b, (k_dec_minus_A<T, false>), g.size, st, gs, u, kap, g,
                inv_h2, out);
}
void launch_res_encode(const double* f, const double* u, const double* kap, const Geom& g, double inv_h2,
                       const SecRef& s, int* nonfinite, double* mon, hipStream_t st) {
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  const double b = (2.0 + (kap ? 1.0 : 0.0)) * g.size * 8.0 + sec_bytes(s);
  if (kap != nullptr)
    CMG_TLAUNCH("k_res_encode", b, k_res_encode<true>, limit, st, f, u, kap, g, inv_h2, s, nonfinite, mon);
  else
    CMG_TLAUNCH("k_res_encode", b, k_res_encode<false>, limit, st, f, u, kap, g, inv_h2, s, nonfinite, mon);
}
template <typename T>
void launch_prolong(const T* coarse, const Geom& gf, const Geom& gc, T* fine, hipStream_t st) {
  if (gf.dim == 3 && gf.level <= 10)
    CMG_TLAUNCH(tname("k_prolong", TName<T>::s).c_str(), (gf.size + gc.size) * sizeof(T), k_prolong3<T>, gf.size, st,
                coarse, gf.level, fine);
  else
    CMG_TLAUNCH(tname("k_prolong", TName<T>::s).c_str(), (gf.size + gc.size) * sizeof(T), k_prolong<T>, gf.size, st,
                coarse, gf, gc, fine);
}
void launch_prolong_add_dec(const SecRef& s, const double* coarse, const Geom& gf, const Geom& gc, double* out,
                            hipStream_t st) {
  CMG_TLAUNCH("k_prolong_add_dec", sec_bytes(s) + 8.0 * (gf.size + gc.size), k_prolong_add_dec, gf.size, st, s,
              coarse, gf, gc, out);
}
template <typename T>
void launch_restrict(const T* fine, const Geom& gc, const Geom& gf, T* coarse, hipStream_t st) {
  CMG_TLAUNCH(tname("k_restrict", TName<T>::s).c_str(), (gf.size + gc.size) * sizeof(T), k_restrict<T>, gc.size,
              st, fine, gc, gf, coarse);
}
template <typename T>
void launch_restrict_encode(const T* fine, const Geom& gc, const Geom& gf, const SecRef& s, int* nonfinite,
                            hipStream_t st) {
  const int64_t limit = ((s.n + s.B - 1) / s.B) * s.B;
  CMG_TLAUNCH(tname("k_restrict_encode", TName<T>::s).c_str(), gf.size * sizeof(T) + sec_bytes(s),
              k_restrict_encode<T>, limit, st, fine, gc, gf, s, nonfinite);
}
template <typename T>
void launch_jacobi(const T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, T omega, T* ynew,
                   hipStream_t st) {
  const double b = (3.0 + (kap ? 1.0 : 0.0)) * g.size * sizeof(T);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_jacobi", TName<T>::s).c_str(), b, (k_jacobi<T, true>), g.size, st, y, rhs, kap, g, inv_h2,
                cpois, omega, ynew);
  else
    CMG_TLAUNCH(tname("k_jacobi", TName<T>::s).c_str(), b, (k_jacobi<T, false>), g.size, st, y, rhs, kap, g, inv_h2,
                cpois, omega, ynew);
}
template <typename T>
void launch_rbgs(T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, int colour, hipStream_t st) {
  // reads y everywhere and rhs on one colour, writes y on one colour
  const double b = (2.0 + (kap ? 1.0 : 0.0)) * g.size * sizeof(T);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_rbgs", TName<T>::s).c_str(), b, (k_rbgs<T, true>), g.size / 2, st, y, rhs, kap, g, inv_h2,
                cpois, colour);
  else
    CMG_TLAUNCH(tname("k_rbgs", TName<T>::s).c_str(), b, (k_rbgs<T, false>), g.size / 2, st, y, rhs, kap, g, inv_h2,
                cpois, colour);
}
template <typename T>
void launch_rbgs_zero(T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, hipStream_t st) {
  const double b = (2.0 + (kap ? 1.0 : 0.0)) * g.size * sizeof(T);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_rbgs_zero", TName<T>::s).c_str(), b, (k_rbgs_zero<T, true>), g.size, st, y, rhs, kap, g,
                inv_h2, cpois);
  else
    CMG_TLAUNCH(tname("k_rbgs_zero", TName<T>::s).c_str(), b, (k_rbgs_zero<T, false>), g.size, st, y, rhs, kap, g,
                inv_h2, cpois);
}
template <typename T>
bool launch_rbgs_sweep(const T* yin, const SecRef* ysec, T* yout, const T* rhs, const T* kap, const Geom& g, T inv_h2,
                       T cpois, bool zero, hipStream_t st) {
  if (g.dim != 3 || g.n < kSwTX) return false;
  const int tiles = (g.n / kSwTX) * (g.n / kSwTY);
  int tz = g.n;  // chunks: at least 4096 workgroups where the level allows
  while (tz > 4 && static_cast<int64_t>(tiles) * (g.n / tz) < 4096) tz >>= 1;
  const dim3 grid(static_cast<unsigned>(tiles * (g.n / tz))), block(kSwNT);
  const double bytes = ((zero ? 2.0 : 3.0) + (kap ? 1.0 : 0.0)) * g.size * sizeof(T);
  const std::string name = tname("k_rbgs_sweep", TName<T>::s);
  const SecRef ys = ysec != nullptr ? *ysec : SecRef{};
#define CMG_SW(D_, Z_, S_)                                                                                      \
  do {                                                                                                          \
    if (g_timing != nullptr) g_timing->begin(name.c_str(), bytes, st);                                          \
    hipLaunchKernelGGL((k_rbgs_sweep<T, D_, Z_, S_>), grid, block, 0, st, yin, ys, yout, rhs, kap, g, inv_h2,    \
                       cpois, tz);                                                                              \
    if (g_timing != nullptr) g_timing->end(st);                                                                 \
  } while (0)
  if (kap != nullptr) {
    if (zero) CMG_SW(true, true, false);
    else if (ysec != nullptr) CMG_SW(true, false, true);
    else CMG_SW(true, false, false);
  } else {
    if (zero) CMG_SW(false, true, false);
    else if (ysec != nullptr) CMG_SW(false, false, true);
    else CMG_SW(false, false, false);
  }
#undef CMG_SW
  return true;
}
template <typename T>
void launch_add(const T* a, const T* b, T* out, int64_t n, hipStream_t st) {
  CMG_TLAUNCH(tname("k_add", TName<T>::s).c_str(), 3.0 * n * sizeof(T), k_add<T>, n, st, a, b, out, n);
}
template <typename T>
void launch_fill(T* x, T v, int64_t n, hipStream_t st) {
  CMG_TLAUNCH(tname("k_fill", TName<T>::s).c_str(), 1.0 * n * sizeof(T), k_fill<T>, n, st, x, v, n);
}
template <typename S, typename D>
void launch_convert(const S* a, D* b, int64_t n, hipStream_t st) {
  CMG_TLAUNCH((std::string("k_convert<") + TName<S>::s + "," + TName<D>::s + ">").c_str(),
              1.0 * n * (sizeof(S) + sizeof(D)), (k_convert<S, D>), n, st, a, b, n);
}
void launch_inject(const double* full, int L, const Geom& g, double* out, hipStream_t st) {
  CMG_TLAUNCH("k_inject", 16.0 * g.size, k_inject, g.size, st, full, L, g, out);
}
void launch_to_full(const double* pad, const Geom& g, double* full, hipStream_t st) {
  const int64_t N = g.n + 1;
  const int64_t tot = g.dim == 3 ? N * N * N : N * N;
  CMG_TLAUNCH("k_to_full", 8.0 * (g.size + tot), k_to_full, tot, st, pad, g, full);
}
void launch_coarse_single(const double* gin, const double* kap, const Geom& g, double inv_h2, double* y,
                          hipStream_t st) {
  if (g_timing != nullptr) g_timing->begin("k_coarse_single", 16.0 * g.size, st);
  hipLaunchKernelGGL(k_coarse_single, dim3(1), dim3(64), 0, st, gin, kap, g, inv_h2, y);
  if (g_timing != nullptr) g_timing->end(st);
}
void launch_coarsen_kappa(const double* fine, const Geom& gc, const Geom& gf, double* coarse, hipStream_t st) {
  CMG_TLAUNCH("k_coarsen_kappa", 8.0 * (gf.size + gc.size), k_coarsen_kappa, gc.size, st, fine, gc, gf, coarse);
}
void launch_check_positive(const double* x, int64_t n, int* flags, hipStream_t st) {
  CMG_TLAUNCH("k_check_positive", 8.0 * n, k_check_positive, n, st, x, n, flags);
}
template <typename T>
void launch_residual_full(const double* f, int Lfull, const double* u, const double* kap, const Geom& g,
                          double inv_h2, T* out, int* nonfinite, double* mon, hipStream_t st) {
  const double b = 8.0 * g.size * (kap != nullptr ? 3.0 : 2.0) + sizeof(T) * static_cast<double>(g.size);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_residual_full", TName<T>::s).c_str(), b, (k_residual_full<T, true>), g.size, st, f, Lfull,
                u, kap, g, inv_h2, out, nonfinite, mon);
  else
    CMG_TLAUNCH(tname("k_residual_full", TName<T>::s).c_str(), b, (k_residual_full<T, false>), g.size, st, f, Lfull,
                u, kap, g, inv_h2, out, nonfinite, mon);
}
template <typename T>
void launch_restrict_residual(const T* r, const T* y, const T* kap, const Geom& gc, const Geom& gf, T inv_h2, T* rc,
                              hipStream_t st) {
  const double b = sizeof(T) * (2.0 * gf.size + gc.size) + (kap != nullptr ? sizeof(T) * gf.size : 0.0);
  if (kap != nullptr)
    CMG_TLAUNCH(tname("k_restrict_residual", TName<T>::s).c_str(), b, (k_restrict_residual<T, true>), gc.size, st, r,
                y, kap, gc, gf, inv_h2, rc);
  else
    CMG_TLAUNCH(tname("k_restrict_residual", TName<T>::s).c_str(), b, (k_restrict_residual<T, false>), gc.size, st, r,
                y, kap, gc, gf, inv_h2, rc);
}
template <typename T>
void launch_prolong_add(const T* coarse, const Geom& gf, const Geom& gc, T* y, hipStream_t st) {
  CMG_TLAUNCH(tname("k_prolong_add", TName<T>::s).c_str(), (2.0 * gf.size + gc.size) * sizeof(T), k_prolong_add<T>,
              gf.size, st, coarse, gf, gc, y);
}
template <typename T>
void launch_add_correction(double* u, const T* y, int64_t n, hipStream_t st) {
  CMG_TLAUNCH(tname("k_add_correction", TName<T>::s).c_str(), (16.0 + sizeof(T)) * n, k_add_correction<T>, n, st, u,
              y, n);
}

void launch_check_finite(const double* x, int64_t n, int* flags, hipStream_t st) {
  CMG_TLAUNCH("k_check_finite", 8.0 * n, k_check_finite, n, st, x, n, flags);
}
void launch_grad_kappa(const double* u, const double* lam, const Geom& gcell, int accumulate, double* grad,
                       hipStream_t st) {
  const double N = gcell.n + 1.0;
  const double nodes = gcell.dim == 3 ? N * N * N : N * N;
  CMG_TLAUNCH("k_grad_kappa", 16.0 * nodes + 8.0 * gcell.size * (accumulate ? 2 : 1), k_grad_kappa, gcell.size, st,
              u, lam, gcell, accumulate, grad);
}
void launch_sumsq(const double* x, int64_t n, double* mon, hipStream_t st) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  if (g_timing != nullptr) g_timing->begin("k_sumsq", 8.0 * n, st);
  hipLaunchKernelGGL(k_sumsq, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, st, x, n, mon);
  if (g_timing != nullptr) g_timing->end(st);
}
void launch_monitor_reset(double* mon, bool entry, hipStream_t st) {
  hipLaunchKernelGGL(k_monitor_reset, dim3(1), dim3(64), 0, st, mon, entry ? 1 : 0);
}
void launch_monitor_check(double* mon, int* flags, int level, double growth, hipStream_t st) {
  hipLaunchKernelGGL(k_monitor_check, dim3(1), dim3(64), 0, st, mon, flags, level, growth);
}

#define CMG_INST_T(T)                                                                                   \
  template void launch_encode<T>(const T*, int64_t, const SecRef&, int*, hipStream_t);                  \
  template void launch_encode_dec<T>(const T*, int64_t, const SecRef&, int*, T*, const T*, const SecRef*,   \
                                     hipStream_t);                                                        \
  template void launch_decode<T>(const SecRef&, int64_t, T*, hipStream_t);                              \
  template void launch_rhs_minus_A<T>(const T*, const T*, const T*, const Geom&, T, T*, hipStream_t);   \
  template void launch_dec_minus_A<T>(const SecRef&, const T*, const T*, const Geom&, T, T*, hipStream_t); \
  template void launch_prolong<T>(const T*, const Geom&, const Geom&, T*, hipStream_t);                 \
  template void launch_restrict<T>(const T*, const Geom&, const Geom&, T*, hipStream_t);                \
  template void launch_restrict_encode<T>(const T*, const Geom&, const Geom&, const SecRef&, int*, hipStream_t); \
  template void launch_jacobi<T>(const T*, const T*, const T*, const Geom&, T, T, T, T*, hipStream_t);  \
  template void launch_rbgs<T>(T*, const T*, const T*, const Geom&, T, T, int, hipStream_t);            \
  template void launch_rbgs_zero<T>(T*, const T*, const T*, const Geom&, T, T, hipStream_t);             \
  template bool launch_rbgs_sweep<T>(const T*, const SecRef*, T*, const T*, const T*, const Geom&, T, T, bool,    \
                                     hipStream_t);                                                              \
  template void launch_add<T>(const T*, const T*, T*, int64_t, hipStream_t);                            \
  template void launch_residual_full<T>(const double*, int, const double*, const double*, const Geom&, double, T*, \
                                        int*, double*, hipStream_t);                                           \
  template void launch_restrict_residual<T>(const T*, const T*, const T*, const Geom&, const Geom&, T, T*,       \
                                            hipStream_t);                                                      \
  template void launch_prolong_add<T>(const T*, const Geom&, const Geom&, T*, hipStream_t);                   \
  template void launch_add_correction<T>(double*, const T*, int64_t, hipStream_t);                            \
  template void launch_fill<T>(T*, T, int64_t, hipStream_t);
CMG_INST_T(float)
CMG_INST_T(double)
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);
template void launch_convert<double, double>(const double*, double*, int64_t, hipStream_t);

}  // namespace cmg
