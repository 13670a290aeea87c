// The V-cycle on the small levels of the hierarchy in one workgroup.
//
// On the smallest levels a kernel launch costs more than the work it does,
// and a V-cycle visits every level with some twenty operations.  Here one
// workgroup of 1024 threads runs the whole down sweep from level Lc, the
// coarsest solve and the up sweep back to Lc, with a workgroup barrier
// between operations.  The level arrays live in LDS (the sections stay in
// global memory); at the end e[Lc] is copied out for the next finer level.
// Each operation computes exactly what the corresponding per-operation
// kernel computes (same expressions in the same order), so the results are
// bit-identical.  A section written here is not read back: the decoded
// values of its new codes go to LDS at the encode (the restricted residual
// of the next coarser level, y' for the up sweep), and the correction
// u' <- Q(dec u' + dec y') runs in the encode of y', on the values its lanes
// hold.  Only the sections from outside (g of the top level, or of every
// level with the restriction chain, and u') are read from global memory.
#include <type_traits>
#include "coarse.h"
#include "timing.h"

namespace cmg {

constexpr int kCoarseNT = 1024;

// (A u) at interior node (i, j, k) of level l (Poisson): the terms and the
// order of apply_A, with 32-bit indices into an LDS level array.  The far
// boundary node (index n) is an implicit 0, read without a branch (the load
// takes the node itself and the value is replaced by 0).
template <int DIM, typename T>
__device__ __forceinline__ T poisson_Au(const T* u, int idx, int i, int j, int k, int l, T ih2) {
  const int n = 1 << l, nn = 1 << (2 * l);
  const bool xo = i + 1 < n, yo = j + 1 < n, zo = k + 1 < n;
  const T up = u[idx];
  const T xm = u[idx - 1], xp = u[xo ? idx + 1 : idx];
  const T ym = u[idx - n], yp = u[yo ? idx + n : idx];
  T s = T(2 * DIM) * up;
  s = s - xm;
  s = s - (xo ? xp : T(0));
  s = s - ym;
  s = s - (yo ? yp : T(0));
  if (DIM == 3) {
    const T zm = u[idx - nn], zp = u[zo ? idx + nn : idx];
    s = s - zm;
    s = s - (zo ? zp : T(0));
  }
  return s * ih2;
}

// DIM and DIFF (variable coefficients) are the problem's: every level of a
// call shares them, so that the index and operator branches fold away.
template <typename T, int DIM, bool DIFF>
__global__ void __launch_bounds__(kCoarseNT) k_coarse_vcycle(CoarseArgs a) {
  constexpr int NW = kCoarseNT / 64;
  __shared__ double pool[kCoarsePoolBytes / 8];
  __shared__ double cpool[3 * kCoarsestMax];
  __shared__ double dense[kDenseWork];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  T* const base = reinterpret_cast<T*>(pool);
  // the five arrays of level l: g, y, z, r, e (in that order)
  auto arr = [&](int l, int which) { return base + a.off[l] + which * static_cast<int>(a.lv[l].g.size); };
  double* const t64 = cpool;
  double* const s64 = cpool + kCoarsestMax;

  auto each = [&](int64_t n, auto&& f) {
    const int m = static_cast<int>(n);
    for (int i = tid; i < m; i += kCoarseNT) f(i);
  };
  // the level's geometry with the dimension as a constant
  auto geo = [&](const CoarseLevel& L) {
    Geom g = L.g;
    g.dim = DIM;
    return g;
  };
  auto kap_of = [&](const CoarseLevel& L) { return DIFF ? static_cast<const T*>(L.kap) : nullptr; };
  auto sync = [&]() { __syncthreads(); };
  auto decode = [&](const SecRef& s, int64_t n, T* x) {
    each(n, [&](int64_t i) { x[i] = static_cast<T>(decode_value(s, i)); });
  };
  auto decode64 = [&](const SecRef& s, int64_t n, double* x) {
    each(n, [&](int64_t i) { x[i] = decode_value(s, i); });
  };
  // One wave per 64 consecutive values (one block of 64 or two of 32).
  // With dec_out, the decoded values of the new codes (as decode() gives
  // them, plus add[i] when add is not null) go to dec_out (which may be x).
  // With u, the section u (same length and block size as s) then takes the
  // correction u <- Q(dec u + dec s) of the same values.
  auto encode = [&](auto* x, int64_t n, const SecRef& s, T* dec_out = nullptr, const T* add = nullptr,
                    const SecRef* u = nullptr) {
    const int64_t limit = limit_of(s);
    for (int64_t base = static_cast<int64_t>(wv) * 64; base < limit; base += NW * 64) {
      const int64_t i = base + lane;
      const double v = (i < n) ? static_cast<double>(x[i]) : 0.0;
      if (a.nonfinite != nullptr && !isfinite(v)) atomicOr(a.nonfinite, 1);
      int e;
      // float input and w <= 24: the float quantiser gives the same codes
      constexpr bool F32 = std::is_same<std::remove_cv_t<std::remove_reference_t<decltype(*x)>>, float>::value;
      const int64_t m = (F32 && s.w <= 24) ? quantise_lane_f32(static_cast<float>(v), s.B, s.w, lane, &e)
                                           : quantise_lane(v, s.B, s.w, &e);
      store_codes_wave(s, base, lane, m, limit);
      if ((lane & (s.B - 1)) == 0 && i < limit) s.exps[blk(s, i)] = static_cast<int16_t>(e);
      // decode_value() of the new code (0 past n: those codes are 0)
      const double d = e == kZeroExp ? 0.0 : ldexp(static_cast<double>(m), e - (s.w - 1));
      if (dec_out != nullptr && i < n) dec_out[i] = add != nullptr ? static_cast<T>(d) + add[i] : static_cast<T>(d);
      if (u != nullptr) {  // u' <- Q(dec u' + dec y')
        const double vu = (i < limit) ? decode_value(*u, i) + d : 0.0;
        int eu;
        const int64_t mu = quantise_lane(vu, u->B, corr_width(*u), &eu);
        store_codes_wave(*u, base, lane, mu, limit);
        if ((lane & (u->B - 1)) == 0 && i < limit) u->exps[blk(*u, i)] = static_cast<int16_t>(eu);
      }
    }
  };
  auto rhs_minus_A = [&](const T* rhs, const T* u, const T* kap, const Geom& g, T ih2, T* out) {
    each(g.size, [&](int idx) {
      int i, j, k;
      unflatten(g, idx, i, j, k);
      T v = T(0);
      if (is_interior(g, i, j, k))
        v = rhs[idx] - (DIFF ? apply_A(u, kap, g, i, j, k, ih2) : poisson_Au<DIM>(u, idx, i, j, k, g.level, ih2));
      out[idx] = v;
    });
  };
  auto restrict_to = [&](const T* fine, const Geom& gc, const Geom& gf, T* coarse) {
    each(gc.size, [&](int idx) {
      int I, J, K;
      unflatten(gc, idx, I, J, K);
      if (!is_interior(gc, I, J, K)) {
        coarse[idx] = T(0);
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
            const int kf = gc.dim == 3 ? 2 * K + oz : 0;
            const T t = static_cast<T>(wz * wy * wx) * fine[flat(gf, 2 * I + ox, 2 * J + oy, kf)];
            s = first ? t : s + t;
            first = false;
          }
        }
      }
      coarse[idx] = s;
    });
  };
  auto prolong = [&](const T* coarse, const Geom& gf, const Geom& gc, T* fine) {
    each(gf.size, [&](int idx) {
      int i, j, k;
      unflatten(gf, idx, i, j, k);
      fine[idx] = prolong_at(coarse, gc, i, j, k);
    });
  };
  auto smooth = [&](const CoarseLevel& L, T* y, const T* rhs, T* scratch, int nu) {
    const T* kap = kap_of(L);
    const T ih2 = static_cast<T>(L.ih2), cp = static_cast<T>(L.cp);
    const Geom g = geo(L);
    if (a.rbgs) {
      for (int s = 0; s < nu; ++s)
        for (int colour = 0; colour < 2; ++colour) {
          // the nodes of one colour: node i = 2 (t mod n/2) + ((j + k + colour) & 1) of row t div (n/2)
          each(g.size >> 1, [&](int t) {
            const int row = t >> (g.level - 1);  // j + n k
            const int j = row & (g.n - 1);
            const int k = g.dim == 3 ? row >> g.level : 0;
            const int i = 2 * (t & ((g.n >> 1) - 1)) + ((j + k + colour) & 1);
            if (!is_interior(g, i, j, k)) return;
            const int idx = (row << g.level) | i;
            const T r = rhs[idx] - (DIFF ? apply_A(y, kap, g, i, j, k, ih2) : poisson_Au<DIM>(y, idx, i, j, k, g.level, ih2));
            const T c = smooth_coeff(kap, g, i, j, k, ih2, cp, T(1));
            y[idx] = y[idx] + c * r;
          });
          sync();
        }
      return;
    }
    const T om = static_cast<T>(a.omega);
    T* p = y;
    T* q = scratch;
    for (int s = 0; s < nu; ++s) {
      each(g.size, [&](int idx) {
        int i, j, k;
        unflatten(g, idx, i, j, k);
        if (!is_interior(g, i, j, k)) {
          q[idx] = T(0);
          return;
        }
        const T r = rhs[idx] - apply_A(p, kap, g, i, j, k, ih2);
        const T c = smooth_coeff(kap, g, i, j, k, ih2, cp, om);
        q[idx] = p[idx] + c * r;
      });
      sync();
      T* t = p;
      p = q;
      q = t;
    }
    if (p != y) {
      each(g.size, [&](int idx) { y[idx] = p[idx]; });
      sync();
    }
  };

  // ---------------------------------------------------------- down sweep
  // g of the top level (of every level with the restriction chain, whose
  // residuals are given) and y = 0 on every level below the coarsest
  for (int l = a.Lc; l > a.lc; --l) {
    if (l == a.Lc || a.chain) decode(a.lv[l].G, a.lv[l].g.size, arr(l, 0));
    T* yf = arr(l, 1);
    each(a.lv[l].g.size, [&](int i) { yf[i] = T(0); });
  }
  sync();
  for (int l = a.Lc; l > a.lc; --l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l - 1];
    T* gf = arr(l, 0);  // dec g, kept for the up sweep
    T* yf = arr(l, 1);  // dec y' after the encode, kept for the up sweep
    T* rf = arr(l, 3);
    smooth(F, yf, gf, arr(l, 4), a.nu_pre);
    encode(yf, F.g.size, F.Y, yf);  // y' = Q(y); yf = dec y'
    sync();
    if (a.chain) continue;  // g_{l-1} is the restricted IR residual, given
    rhs_minus_A(gf, yf, kap_of(F), geo(F), static_cast<T>(F.ih2), rf);
    sync();
    restrict_to(rf, geo(C), geo(F), arr(l - 1, 3));
    sync();
    encode(arr(l - 1, 3), C.g.size, C.G, arr(l - 1, 0));  // g_{l-1} = Q(R r); dec g_{l-1}
    sync();
  }
  // ------------------------------------------------------ coarsest (float64)
  {
    const CoarseLevel& B = a.lv[a.lc];
    decode64(B.G, B.g.size, t64);
    each(B.g.size, [&](int t) { s64[t] = 0.0; });
    sync();
    if (tid == 0) coarse_solve_dense(t64, DIFF ? a.kap64 : nullptr, geo(B), B.ih2, s64, cpool + 2 * kCoarsestMax, dense);
    sync();
    encode(s64, B.g.size, B.Yp, arr(a.lc, 4), nullptr, &B.U);  // y' = Q(A^-1 g); e = dec y'; u' += y'
    sync();
  }
  // ------------------------------------------------------------ up sweep
  for (int l = a.lc + 1; l <= a.Lc; ++l) {
    const CoarseLevel& F = a.lv[l];
    const CoarseLevel& C = a.lv[l - 1];
    const T* gf = arr(l, 0);  // dec g and dec y' from the down sweep
    T* yf = arr(l, 1);
    T* zf = arr(l, 2);
    T* rf = arr(l, 3);
    prolong(arr(l - 1, 4), geo(F), geo(C), zf);
    sync();
    rhs_minus_A(gf, zf, kap_of(F), geo(F), static_cast<T>(F.ih2), rf);
    sync();
    smooth(F, yf, rf, arr(l, 4), a.nu_post);
    // y' = Q(y); e = dec y' + z; u' <- Q(dec u' + dec y')
    encode(yf, F.g.size, F.Yp, l < a.Lp ? arr(l, 4) : nullptr, zf, &F.U);
    sync();
  }
  if (a.Lc < a.Lp) {  // e[Lc] for the next finer level
    const T* e = arr(a.Lc, 4);
    T* out = static_cast<T*>(a.lv[a.Lc].ef);
    each(a.lv[a.Lc].g.size, [&](int i) { out[i] = e[i]; });
  }
}

template <typename T>
void launch_coarse_vcycle(const CoarseArgs& a, hipStream_t st) {
  double bytes = 0.0;  // the sections read and written
  for (int l = a.lc; l <= a.Lc; ++l) bytes += 5.0 * 2.0 * static_cast<double>(a.lv[l].g.size);
  if (g_timing != nullptr) g_timing->begin("k_coarse_vcycle", bytes, st);
  const bool three = a.lv[a.Lc].g.dim == 3, diff = a.lv[a.Lc].kap != nullptr;
  auto kern = three ? (diff ? k_coarse_vcycle<T, 3, true> : k_coarse_vcycle<T, 3, false>)
                    : (diff ? k_coarse_vcycle<T, 2, true> : k_coarse_vcycle<T, 2, false>);
  hipLaunchKernelGGL(kern, dim3(1), dim3(kCoarseNT), 0, st, a);
  if (g_timing != nullptr) g_timing->end(st);
}

template void launch_coarse_vcycle<float>(const CoarseArgs&, hipStream_t);
template void launch_coarse_vcycle<double>(const CoarseArgs&, hipStream_t);

}  // namespace cmg
