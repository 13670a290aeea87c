// Launchers of the fused 3-D level-sweep kernels (fused.hip).  Each returns
// false, launching nothing, when the level is not handled by a fused kernel
// (2-D, or rows shorter than one 64-node tile).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace cmg {

// y'_l = Q(S^nu(0; g_l)), red-black Gauss-Seidel, nu in {1, 2}.
bool fused_down_smooth(const SecRef& G, const SecRef& Y, const Geom& g, int nu, float cp, float ih2, hipStream_t st);

// z = P e_{l-1}; Yp = Q(S^nu(dec Y; g_l - A z)); u'_l = Q(u'_l + dec Yp);
// eout (nullable) = dec Yp + z.  Y (pre-smoothed) is only read: other
// workgroups read it at their halos while Yp is written.  u_zero: U holds
// zeros that were never written (its codes are read as 0).
bool fused_up_smooth(const float* ec, const SecRef& G, const SecRef& Y, const SecRef& Yp, const SecRef& U,
                     float* eout, const Geom& g, const Geom& gc, int nu, float cp, float ih2, hipStream_t st,
                     bool u_zero = false);

// g_{l-1} = Q(R(g_l - A y'_l)).
bool fused_resid_restrict(const SecRef& G, const SecRef& Y, const SecRef& Gc, const Geom& g, const Geom& gc,
                          float ih2, hipStream_t st);

// g = Q(f - A(dec u' + P uc)) in float64; f sampled from the level-Lfull grid.
// sumsq (nullable): the IR residual monitor's slots (device.h), which receive
// sum t^2 (unordered atomics, one per wave).  With Uc (u' of level gc) and
// ucc (the float64 level array one level below gc), the coarse solution is
// rebuilt as dec Uc + P ucc where it is needed and uc is not read.  u_zero:
// U holds zeros that were never written (its codes are read as 0).
bool fused_ir_residual(const SecRef& U, const double* uc, const double* f, int Lfull, const Geom& g, const Geom& gc,
                       double ih2, const SecRef& Gout, int* nonfinite, double* sumsq, hipStream_t st,
                       const SecRef* Uc = nullptr, const double* ucc = nullptr, bool u_zero = false);

// Full node grid u = dec u'_l + P uc (3-D levels of at least 64^3 nodes);
// Uc and ucc as for fused_ir_residual.
bool fused_decode_full(const SecRef& U, const double* uc, const Geom& g, const Geom& gc, double* full,
                       hipStream_t st, const SecRef* Uc = nullptr, const double* ucc = nullptr);

// One decode-chain step u_l = dec u'_l + P u_{l-1} in the padded layout
// (3-D levels of at least 64^3 nodes).
bool fused_decode_level(const SecRef& U, const double* uc, const Geom& g, const Geom& gc, double* out,
                        hipStream_t st);

}  // namespace cmg
