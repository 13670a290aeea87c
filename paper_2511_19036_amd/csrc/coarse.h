// The V-cycle below a given level in a single workgroup (coarse.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace cmg {

constexpr int kCoarseMaxLevel = 7;             // levels 1 .. 7 fit the argument block
constexpr int kCoarsePoolBytes = 112 * 1024;    // LDS for the level arrays (five per level)
constexpr int kCoarsestMax = 64;                // values of the coarsest level (float64 scratch)

// Bytes of the LDS arrays of levels lc .. l for a value size vs.
inline int64_t coarse_pool_bytes(int dim, int lc, int l, int vs) {
  int64_t n = 0;
  for (int k = lc; k <= l; ++k) n += static_cast<int64_t>(1) << (dim * k);
  return 5 * n * vs;
}

struct CoarseLevel {
  SecRef G, Y, Yp, U;                   // widths already set for this cycle
  void* ef;                             // e of the level in the V-cycle type (written for level Lc only)
  const void* kap;                      // cell coefficients in the V-cycle type, or null (Poisson)
  Geom g;
  double ih2;                           // h^-2
  double cp;                            // smoothing coefficient (omega /) (2 d h^-2)
};

struct CoarseArgs {
  CoarseLevel lv[kCoarseMaxLevel + 1];  // indexed by level
  int off[kCoarseMaxLevel + 1];         // offset (values) of each level's arrays in LDS
  const double* kap64;                  // coarsest level coefficients (null for Poisson)
  int lc, Lc, Lp;                       // coarsest level, top level of this call, FMG level
  int nu_pre, nu_post, rbgs;
  int chain;                            // 1: every G is given (Alg. 2 chain, nu_pre = 0); no restriction
  double omega;
  int* nonfinite;
};

// Down sweep Lc .. lc+1 from G[Lc], coarsest solve, up sweep lc+1 .. Lc with
// the corrections of u'; writes e[Lc] when Lc < Lp.  Same operations, order
// and arithmetic as the per-operation kernels.
template <typename T>
void launch_coarse_vcycle(const CoarseArgs& a, hipStream_t st);

}  // namespace cmg
