// Host-side launchers of the level kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace cmg {

template <typename T> void launch_encode(const T* x, int64_t n, const SecRef& s, int* nonfinite, hipStream_t st);
// The encode, and the decoded values of the new codes written to out (plus
// add[i] when add is not null): an encode followed by a decode (and an add)
// in one pass.  out may be x.  With correct_u (a section with the blocks of
// s), also u <- Q(dec u + dec s), as launch_correct does.
template <typename T>
void launch_encode_dec(const T* x, int64_t n, const SecRef& s, int* nonfinite, T* out, const T* add,
                       const SecRef* correct_u, hipStream_t st);
template <typename T> void launch_decode(const SecRef& s, int64_t n, T* x, hipStream_t st);
void launch_widen(const SecRef& s, int k, hipStream_t st);
// Encode the interior of a full node array (boundary and far nodes 0).
void launch_encode_full(const double* full, int L, const Geom& g, const SecRef& s, int* nonfinite, hipStream_t st);
void launch_zero_section(const SecRef& s, hipStream_t st);
void launch_correct(const SecRef& u, const SecRef& y, hipStream_t st);

template <typename T>
void launch_rhs_minus_A(const T* rhs, const T* u, const T* kap, const Geom& g, T inv_h2, T* out, hipStream_t st);
// s = Q(f - A u) in float64 (interior; 0 on the boundary): the residual of
// iterative refinement and its encode in one pass (flags non-finite values
// in *nonfinite like launch_encode).
void launch_res_encode(const double* f, const double* u, const double* kap, const Geom& g, double inv_h2,
                       const SecRef& s, int* nonfinite, double* mon, hipStream_t st);
// out = dec(gs) - A u (interior; 0 on the boundary): a decode of the
// right-hand side section and launch_rhs_minus_A in one pass.
template <typename T>
void launch_dec_minus_A(const SecRef& gs, const T* u, const T* kap, const Geom& g, T inv_h2, T* out, hipStream_t st);
template <typename T> void launch_prolong(const T* coarse, const Geom& gf, const Geom& gc, T* fine, hipStream_t st);
void launch_prolong_add_dec(const SecRef& s, const double* coarse, const Geom& gf, const Geom& gc, double* out,
                            hipStream_t st);
template <typename T> void launch_restrict(const T* fine, const Geom& gc, const Geom& gf, T* coarse, hipStream_t st);
// s = Q(R fine): the restriction and the encode of its result in one pass.
template <typename T>
void launch_restrict_encode(const T* fine, const Geom& gc, const Geom& gf, const SecRef& s, int* nonfinite,
                            hipStream_t st);
template <typename T>
void launch_jacobi(const T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, T omega, T* ynew,
                   hipStream_t st);
template <typename T>
void launch_rbgs(T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, int colour, hipStream_t st);
// The first red half-sweep from y = 0, writing all of y (the other nodes 0):
// the same values as filling y with zeros and running launch_rbgs(colour 0).
template <typename T>
void launch_rbgs_zero(T* y, const T* rhs, const T* kap, const Geom& g, T inv_h2, T cpois, hipStream_t st);
// One red-black Gauss-Seidel sweep (red then black) of a 3-D level with at
// least 64 nodes per axis in one launch, out of place (yin -> yout; with
// zero, y is taken as 0, and with ysec not null, y is the decoded section;
// then yin is not read).  The same values as the two launch_rbgs
// half-sweeps.  Returns false (nothing launched) for other levels.
template <typename T>
bool launch_rbgs_sweep(const T* yin, const SecRef* ysec, T* yout, const T* rhs, const T* kap, const Geom& g, T inv_h2,
                       T cpois, bool zero, hipStream_t st);
template <typename T> void launch_add(const T* a, const T* b, T* out, int64_t n, hipStream_t st);
// Plain FP64 multigrid: out = (T)(f - A u) with f sampled from the finest
// node array (monitor slots and non-finite flag fed); rc = R (r - A y);
// y += P yc in place; u += (double) y.
template <typename T>
void launch_residual_full(const double* f, int Lfull, const double* u, const double* kap, const Geom& g,
                          double inv_h2, T* out, int* nonfinite, double* mon, hipStream_t st);
template <typename T>
void launch_restrict_residual(const T* r, const T* y, const T* kap, const Geom& gc, const Geom& gf, T inv_h2, T* rc,
                              hipStream_t st);
template <typename T> void launch_prolong_add(const T* coarse, const Geom& gf, const Geom& gc, T* y, hipStream_t st);
template <typename T> void launch_add_correction(double* u, const T* y, int64_t n, hipStream_t st);
template <typename T> void launch_fill(T* x, T v, int64_t n, hipStream_t st);
template <typename S, typename D> void launch_convert(const S* a, D* b, int64_t n, hipStream_t st);

void launch_inject(const double* full, int L, const Geom& g, double* out, hipStream_t st);
void launch_to_full(const double* pad, const Geom& g, double* full, hipStream_t st);
void launch_coarse_single(const double* gin, const double* kap, const Geom& g, double inv_h2, double* y,
                          hipStream_t st);
void launch_coarsen_kappa(const double* fine, const Geom& gc, const Geom& gf, double* coarse, hipStream_t st);
void launch_check_positive(const double* x, int64_t n, int* flags, hipStream_t st);
void launch_check_finite(const double* x, int64_t n, int* flags, hipStream_t st);
void launch_grad_kappa(const double* u, const double* lam, const Geom& gcell, int accumulate, double* grad,
                       hipStream_t st);
// Sum of squares of x into the IR residual monitor's slots (device.h).
void launch_sumsq(const double* x, int64_t n, double* mon, hipStream_t st);
void launch_monitor_reset(double* mon, bool entry, hipStream_t st);
void launch_monitor_check(double* mon, int* flags, int level, double growth, hipStream_t st);

}  // namespace cmg
