// Solver context, FMG / V-cycle orchestration and the C ABI of cmg.h.
//
// Compact FMG (Alg. 3): coarsest solve; per FMG level widen the coarser
// solution sections and append a zero section; N times: IR residual from the
// decoded solution (Alg. 2, float64), one compact V-cycle from a zero
// correction (Alg. 1 with nu_pre / nu_post sweeps, arithmetic type T), and
// the section-wise correction u' += y' (float64).  Plain FMG (Alg. SM2)
// keeps float64 standard vectors and a correction-scheme V-cycle.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <type_traits>
#include <vector>

#include "abfp.h"
#include "cmg.h"
#include "coarse.h"
#include "fused.h"
#include "launch.h"
#include "timing.h"

using namespace cmg;

namespace {

struct CmgError {
  cmg_status code;
  std::string msg;
};

thread_local std::string g_thread_error;

[[noreturn]] void fail(cmg_status code, const std::string& msg) { throw CmgError{code, msg}; }

#define HIPCK(call)                                                                                \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess)                                                                          \
      fail(e_ == hipErrorOutOfMemory ? CMG_ERR_OUT_OF_MEMORY : CMG_ERR_HIP,                        \
           std::string(#call) + ": " + hipGetErrorString(e_));                                     \
  } while (0)
#define KCK() HIPCK(hipGetLastError())

int container_bits(int w) {
  if (w <= 8) return 8;
  if (w <= 12) return 12;
  if (w <= 16) return 16;
  if (w <= 32) return 32;
  return 64;
}

int64_t n_blocks(int64_t n, int B) { return (n + B - 1) / B; }
int64_t code_bytes(int64_t n, int B, int w) { return n_blocks(n, B) * B * container_bits(w) / 8; }

enum MemCat { kSections = 0, kCoarse64, kCoarseWork, kFineWork, kKappa, kOther, kNumCat };

struct Section {
  void* codes = nullptr;
  int16_t* exps = nullptr;
  int64_t n = 0, nblk = 0, bytes = 0;
  // w: width of the stored codes (what decoding uses); wt: the section's
  // width on the current FMG level (u' only: raised on entering a level,
  // reached by the codes at the section's next correction, or by widening
  // them when they are exported)
  int B = 64, w = 2, wt = 2, cbits = 8;
  SecRef ref() const { return SecRef{codes, exps, n, B, w, cbits}; }
  // for a correction u <- Q(dec u + dec y): new codes of width wt
  SecRef ref_corr() const {
    SecRef r = ref();
    r.wq = wt;
    return r;
  }
  void set_w(int bits) { w = wt = bits; }
};

struct LevelData {
  Geom g{};
  Section U, G, Y;                    // compact sections u', g = r - s, pre-smoothed y'
  // Post-smoothed y' (the correction added to u').  A section of its own only
  // with keep_correction; otherwise the buffers of Y where the up sweep runs
  // one kernel per operation (Y has been read before y' is rounded), and no
  // buffers at all under the fused up sweep, which never stores it.
  Section Yp;
  void *gf = nullptr, *yf = nullptr;  // V-cycle arrays in the arithmetic type T
  void *zf = nullptr, *rf = nullptr, *ef = nullptr;
  double* uh = nullptr;   // decoded solution (compact) / solution (plain)
  double* t64 = nullptr;  // float64 residual
  double* f64 = nullptr;  // injected right-hand side
  double* s64 = nullptr;  // float64 scratch (coarse solve)
  double* kap64 = nullptr;
  void* kapT = nullptr;
  // u' of a new FMG level is zero: where the fused IR residual and up sweep
  // are its first readers, they read its codes as 0 and the zero fill is
  // left out until another reader needs it (ensure_u)
  bool u_zero = false;
};

double inv_h2(int level) { return std::ldexp(1.0, 2 * level); }

}  // namespace

struct cmg_ctx_s {
  cmg_problem p{};
  cmg_opts o{};
  hipStream_t st = nullptr;
  std::vector<LevelData> lv;
  std::vector<void*> allocs;
  int64_t mem[kNumCat] = {};
  int Lp = -1;
  int* flags = nullptr;   // [0] non-positive kappa, [1] non-finite value, [2] FMG level that diverged
  double* mon = nullptr;  // IR residual monitor (device.h: slots, smallest and last sum of squares)
  double* pu[2] = {nullptr, nullptr};  // plain path: float64 FMG solution, levels L, L-2, ... / L-1, L-3, ...
  bool mon_fresh = true;  // the next IR residual is the first one on its FMG level
  bool dead = false;
  bool timing_on = false;
  KernelTiming timing;
  std::string err;

  void* alloc(size_t bytes, MemCat cat) {
    void* ptr = nullptr;
    if (bytes == 0) return nullptr;
    HIPCK(hipMalloc(&ptr, bytes));
    allocs.push_back(ptr);
    mem[cat] += static_cast<int64_t>(bytes);
    return ptr;
  }
  int lc() const { return p.coarsest; }
  int cap_ry() const { return o.vcycle_prec == CMG_FP32 ? 24 : 53; }
  int wu(int l, int Lp_) const { return std::min(53, o.bits_u + o.inc_u * (Lp_ - l)); }
  int wr(int l, int Lp_) const { return std::min(cap_ry(), o.bits_r + o.inc_ry * (Lp_ - l)); }
  int wy(int l, int Lp_) const { return std::min(cap_ry(), o.bits_y + o.inc_ry * (Lp_ - l)); }
  int64_t full_size(int level) const {
    int64_t N = (int64_t{1} << level) + 1;
    return p.dim == 3 ? N * N * N : N * N;
  }
  bool compact() const { return o.storage == CMG_COMPACT_BFP; }
  // Without pre-smoothing (V(0, nu2)) the V-cycle takes the residual of
  // every level from the IR residual: Alg. 2 restricts the unrounded float64
  // residual level by level and rounds each level once.
  bool chain() const { return compact() && o.nu_pre == 0; }
  // Levels handled by the fused 3-D kernels (rows of at least 64 nodes).
  bool fused3d() const {
    return compact() && p.dim == 3 && p.op == CMG_POISSON && o.smoother == CMG_RBGS &&
           o.vcycle_prec == CMG_FP32 && o.nu_pre >= 0 && o.nu_pre <= 2 && o.nu_post >= 1 && o.nu_post <= 2;
  }
  bool smooth_fused(int l) const { return fused3d() && l >= 6; }
  bool rr_fused(int l) const { return fused3d() && l >= 7; }
  bool res_fused(int l) const { return compact() && p.dim == 3 && p.op == CMG_POISSON && l >= 6 && !chain(); }
  // The fused IR residual and final decode of level l rebuild the decoded
  // solution of level l - 1 from its section and the level below (the
  // multi-level sweep of the decode chain), so that u_{l-1} is never stored:
  // the chain of decoded levels ends at l - 2.
  bool skip_fused(int l) const { return res_fused(l) && l - 2 >= lc(); }
  // u' of a new FMG level l is read first by the fused IR residual and up
  // sweep, which take it as zero without the fill
  bool u_lazy(int l) const { return smooth_fused(l) && res_fused(l); }
};

namespace {

Geom make_geom(int dim, int level) {
  Geom g;
  g.dim = dim;
  g.level = level;
  g.n = 1 << level;
  g.size = int64_t{1} << (dim * level);
  return g;
}

// ------------------------------------------------------------ validation
void validate(const cmg_problem* p, const cmg_opts* o) {
  if (p == nullptr || o == nullptr) fail(CMG_ERR_INVALID_ARG, "problem and options must not be NULL");
  if (p->dim != 2 && p->dim != 3) fail(CMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  const int maxL = p->dim == 3 ? 10 : 14;
  if (p->L < 2 || p->L > maxL) fail(CMG_ERR_INVALID_ARG, "L out of range");
  if (p->coarsest < 1 || p->coarsest >= p->L) fail(CMG_ERR_INVALID_ARG, "need 1 <= coarsest < L");
  if (p->coarsest > 2)
    fail(CMG_ERR_UNSUPPORTED, "coarsest levels 1 and 2 (a dense solve of at most 27 interior nodes) are implemented");
  if (p->op != CMG_POISSON && p->op != CMG_DIFFUSION) fail(CMG_ERR_INVALID_ARG, "unknown operator");
  if (p->batch < 1) fail(CMG_ERR_INVALID_ARG, "batch must be >= 1");
  if (o->smoother != CMG_WJACOBI && o->smoother != CMG_RBGS) fail(CMG_ERR_INVALID_ARG, "unknown smoother");
  if (o->smoother == CMG_WJACOBI && !(o->omega > 0.0 && o->omega < 2.0))
    fail(CMG_ERR_INVALID_ARG, "omega must lie in (0, 2)");
  if (o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre > 16 || o->nu_post > 16)
    fail(CMG_ERR_INVALID_ARG, "smoothing sweeps must lie in [0, 16]");
  if (o->ir_iters < 1 || o->ir_iters > 64) fail(CMG_ERR_INVALID_ARG, "ir_iters must lie in [1, 64]");
  if (o->final_iters < 0 || o->final_iters > 200) fail(CMG_ERR_INVALID_ARG, "final_iters must lie in [0, 200]");
  if (o->vcycles != 1) fail(CMG_ERR_UNSUPPORTED, "vcycles (nu) must be 1: the V-cycle starts from zero");
  if (o->storage != CMG_PLAIN_FP64 && o->storage != CMG_COMPACT_BFP) fail(CMG_ERR_INVALID_ARG, "unknown storage");
  if (o->vcycle_prec != CMG_FP32 && o->vcycle_prec != CMG_FP64) fail(CMG_ERR_INVALID_ARG, "unknown vcycle_prec");
  if (o->storage == CMG_COMPACT_BFP) {
    const int cap = o->vcycle_prec == CMG_FP32 ? 24 : 53;
    if (o->bfp_block != 32 && o->bfp_block != 64) fail(CMG_ERR_INVALID_ARG, "bfp_block must be 32 or 64");
    if (o->bits_u < 2 || o->bits_u > 53) fail(CMG_ERR_INVALID_ARG, "bits_u must lie in [2, 53]");
    if (o->bits_r < 2 || o->bits_r > cap || o->bits_y < 2 || o->bits_y > cap)
      fail(CMG_ERR_INVALID_ARG, "bits_r / bits_y must lie in [2, 24] (FP32 V-cycle) or [2, 53]");
    if (o->inc_u < 0 || o->inc_ry < 0 || o->inc_u > 8 || o->inc_ry > 8)
      fail(CMG_ERR_INVALID_ARG, "increments must lie in [0, 8]");
  }
  if (o->keep_correction != 0 && o->keep_correction != 1) fail(CMG_ERR_INVALID_ARG, "keep_correction must be 0 or 1");
}

// ------------------------------------------------------------ setup
void alloc_section(cmg_ctx c, Section& s, const Geom& g, int wmax) {
  s.n = g.size;
  s.B = c->o.bfp_block;
  s.nblk = n_blocks(s.n, s.B);
  s.cbits = container_bits(wmax);
  s.set_w(wmax);
  s.bytes = code_bytes(s.n, s.B, wmax);
  // 16 bytes of padding: the fused kernels read codes as 8-byte windows
  s.codes = c->alloc(static_cast<size_t>(s.bytes) + 16, kSections);
  s.exps = static_cast<int16_t*>(c->alloc(static_cast<size_t>(s.nblk) * 2, kSections));
}

void setup_levels(cmg_ctx c, const double* kappa) {
  const int L = c->p.L, lc = c->lc(), d = c->p.dim;
  const size_t tsz = c->o.vcycle_prec == CMG_FP32 ? 4 : 8;
  c->lv.resize(L + 1);
  for (int l = lc; l <= L; ++l) {
    LevelData& D = c->lv[l];
    D.g = make_geom(d, l);
    const size_t n = static_cast<size_t>(D.g.size);
    const MemCat work = l == L ? kFineWork : kCoarseWork;
    const MemCat f64c = l == L ? kFineWork : kCoarse64;
    if (c->compact()) {
      alloc_section(c, D.U, D.g, c->wu(l, L));
      alloc_section(c, D.G, D.g, c->wr(l, L));
      alloc_section(c, D.Y, D.g, c->wy(l, L));
      if (c->o.keep_correction) {
        alloc_section(c, D.Yp, D.g, c->wy(l, L));
      } else {
        D.Yp = D.Y;
        if (c->smooth_fused(l)) D.Yp.codes = D.Yp.exps = nullptr;
      }
      // per-operation scratch only where a per-operation kernel runs
      const bool v1s = !c->smooth_fused(l), v1rr = !c->rr_fused(l);
      const bool target = l < L && !c->rr_fused(l + 1);  // restriction target of level l + 1
      if (v1s || v1rr) {
        D.gf = c->alloc(n * tsz, work);
        D.yf = c->alloc(n * tsz, work);
      }
      if (v1s || v1rr || target) D.rf = c->alloc(n * tsz, work);
      if (v1s) D.zf = c->alloc(n * tsz, work);
      if (l < L || v1s) D.ef = c->alloc(n * tsz, work);
      const bool v1res = !c->res_fused(l);
      const bool rebuilt = l == L - 1 && c->skip_fused(L);  // u_{L-1} is rebuilt where it is read
      if ((l < L && !rebuilt) || d == 2 || v1res) D.uh = static_cast<double*>(c->alloc(n * 8, f64c));
      if (v1res || l == lc || (c->chain() && l < L)) D.t64 = static_cast<double*>(c->alloc(n * 8, f64c));
      if (v1res || l == lc) D.f64 = static_cast<double*>(c->alloc(n * 8, f64c));
    } else {
      // u, r and y per level (the V-cycle runs in place, with fused
      // residual-restriction and prolongation-add kernels); weighted Jacobi
      // needs a second y array, and so do the one-launch red-black sweeps
      // of 3-D levels from 64^3 (out of place: a workgroup's halo must not
      // see its neighbours' new values); the float64 solution of the
      // current FMG level lives in pu[(L - level) & 1]
      D.yf = c->alloc(n * tsz, work);
      D.rf = c->alloc(n * tsz, work);
      if (c->o.smoother == CMG_WJACOBI || (d == 3 && D.g.n >= 64)) D.zf = c->alloc(n * tsz, work);
      if (l == lc) {
        D.t64 = static_cast<double*>(c->alloc(n * 8, kCoarse64));
        D.f64 = static_cast<double*>(c->alloc(n * 8, kCoarse64));
      }
    }
    if (l == lc) D.s64 = static_cast<double*>(c->alloc(n * 8, kCoarse64));
  }
  if (!c->compact()) {
    c->pu[0] = static_cast<double*>(c->alloc(static_cast<size_t>(c->lv[L].g.size) * 8, kFineWork));
    c->pu[1] = static_cast<double*>(c->alloc(static_cast<size_t>(c->lv[L - 1].g.size) * 8, kCoarse64));
  }
  c->flags = static_cast<int*>(c->alloc(64, kOther));
  c->mon = static_cast<double*>(c->alloc(kMonDoubles * 8, kOther));
  HIPCK(hipMemsetAsync(c->flags, 0, 64, c->st));
  if (c->p.op == CMG_DIFFUSION) {
    for (int l = lc; l <= L; ++l) {
      LevelData& D = c->lv[l];
      const size_t n = static_cast<size_t>(D.g.size);
      D.kap64 = static_cast<double*>(c->alloc(n * 8, kKappa));
      D.kapT = tsz == 4 ? c->alloc(n * 4, kKappa) : D.kap64;
    }
    LevelData& F = c->lv[L];
    HIPCK(hipMemcpyAsync(F.kap64, kappa, static_cast<size_t>(F.g.size) * 8, hipMemcpyDeviceToDevice, c->st));
    launch_check_positive(F.kap64, F.g.size, c->flags, c->st);
    KCK();
    int h[2] = {0, 0};
    HIPCK(hipMemcpyAsync(h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->st));
    HIPCK(hipStreamSynchronize(c->st));
    if (h[1]) fail(CMG_ERR_NONFINITE, "kappa holds NaN or Inf");
    if (h[0]) fail(CMG_ERR_INVALID_ARG, "kappa must be positive");
    for (int l = L - 1; l >= lc; --l) {
      launch_coarsen_kappa(c->lv[l + 1].kap64, c->lv[l].g, c->lv[l + 1].g, c->lv[l].kap64, c->st);
      KCK();
    }
    if (tsz == 4)
      for (int l = lc; l <= L; ++l) {
        launch_convert<double, float>(c->lv[l].kap64, static_cast<float*>(c->lv[l].kapT), c->lv[l].g.size, c->st);
        KCK();
      }
  }
  HIPCK(hipStreamSynchronize(c->st));
}

// ------------------------------------------------------------ V-cycle pieces
template <typename T>
const T* kapT(cmg_ctx c, int l) {
  return c->p.op == CMG_DIFFUSION ? static_cast<const T*>(c->lv[l].kapT) : nullptr;
}
const double* kap64(cmg_ctx c, int l) { return c->p.op == CMG_DIFFUSION ? c->lv[l].kap64 : nullptr; }

// nu sweeps of the smoother on A y = rhs (level l), in place on y.  Without
// a scratch array red-black Gauss-Seidel runs one launch per half-sweep.
template <typename T>
void smooth(cmg_ctx c, int l, T* y, const T* rhs, T* scratch, int nu) {
  LevelData& D = c->lv[l];
  const double ih2 = inv_h2(l);
  const T* kap = kapT<T>(c, l);
  const int d = c->p.dim;
  if (c->o.smoother == CMG_RBGS) {
    const T cp = static_cast<T>(1.0 / (2.0 * d * ih2));
    if (nu > 0 && d == 3 && D.g.n >= 64 && scratch != nullptr) {  // one launch per sweep, out of place
      T* a = y;
      T* b = scratch;
      for (int s = 0; s < nu; ++s) {
        launch_rbgs_sweep<T>(a, nullptr, b, rhs, kap, D.g, static_cast<T>(ih2), cp, false, c->st);
        KCK();
        std::swap(a, b);
      }
      if (a != y) HIPCK(hipMemcpyAsync(y, a, static_cast<size_t>(D.g.size) * sizeof(T), hipMemcpyDeviceToDevice, c->st));
      return;
    }
    for (int s = 0; s < nu; ++s)
      for (int colour = 0; colour < 2; ++colour) {
        launch_rbgs<T>(y, rhs, kap, D.g, static_cast<T>(ih2), cp, colour, c->st);
        KCK();
      }
    return;
  }
  const T cp = static_cast<T>(c->o.omega / (2.0 * d * ih2));
  const T om = static_cast<T>(c->o.omega);
  T* a = y;
  T* b = scratch;
  for (int s = 0; s < nu; ++s) {
    launch_jacobi<T>(a, rhs, kap, D.g, static_cast<T>(ih2), cp, om, b, c->st);
    KCK();
    std::swap(a, b);
  }
  if (a != y)  // odd number of sweeps: the result sits in the scratch array
    HIPCK(hipMemcpyAsync(y, a, static_cast<size_t>(D.g.size) * sizeof(T), hipMemcpyDeviceToDevice, c->st));
}

// nu sweeps of the smoother from y = 0 (y is overwritten).  Red-black
// Gauss-Seidel starts with a pointwise red half-sweep that writes all of y.
template <typename T>
void smooth_from_zero(cmg_ctx c, int l, T* y, const T* rhs, T* scratch, int nu) {
  LevelData& D = c->lv[l];
  if (c->o.smoother != CMG_RBGS || nu < 1) {
    launch_fill<T>(y, T(0), D.g.size, c->st);
    KCK();
    smooth<T>(c, l, y, rhs, scratch, nu);
    return;
  }
  const double ih2 = inv_h2(l);
  const T* kap = kapT<T>(c, l);
  const T cp = static_cast<T>(1.0 / (2.0 * c->p.dim * ih2));
  if (c->p.dim == 3 && D.g.n >= 64 && scratch != nullptr) {  // one launch per sweep, the first from zero
    T* a = (nu & 1) ? scratch : y;
    T* b = (nu & 1) ? y : scratch;
    for (int s = 0; s < nu; ++s) {
      launch_rbgs_sweep<T>(a, nullptr, b, rhs, kap, D.g, static_cast<T>(ih2), cp, s == 0, c->st);
      KCK();
      std::swap(a, b);
    }
    return;
  }
  launch_rbgs_zero<T>(y, rhs, kap, D.g, static_cast<T>(ih2), cp, c->st);
  launch_rbgs<T>(y, rhs, kap, D.g, static_cast<T>(ih2), cp, 1, c->st);
  KCK();
  smooth<T>(c, l, y, rhs, scratch, nu - 1);
}

// nu sweeps of the smoother starting from the decoded section ys (written
// to y).  With one launch per sweep the first sweep reads the codes itself.
template <typename T>
void smooth_from_section(cmg_ctx c, int l, const SecRef& ys, T* y, const T* rhs, T* scratch, int nu) {
  LevelData& D = c->lv[l];
  if (c->o.smoother == CMG_RBGS && nu >= 1 && c->p.dim == 3 && D.g.n >= 64) {
    const double ih2 = inv_h2(l);
    const T* kap = kapT<T>(c, l);
    const T cp = static_cast<T>(1.0 / (2.0 * c->p.dim * ih2));
    T* a = (nu & 1) ? scratch : y;  // the last sweep writes y
    T* b = (nu & 1) ? y : scratch;
    for (int s = 0; s < nu; ++s) {
      launch_rbgs_sweep<T>(a, s == 0 ? &ys : nullptr, b, rhs, kap, D.g, static_cast<T>(ih2), cp, false, c->st);
      KCK();
      std::swap(a, b);
    }
    return;
  }
  launch_decode<T>(ys, D.g.size, y, c->st);
  KCK();
  smooth<T>(c, l, y, rhs, scratch, nu);
}

// Write the zeros of a u' section that the fused kernels took as zero.
void ensure_u(cmg_ctx c, int l) {
  LevelData& D = c->lv[l];
  if (!D.u_zero) return;
  launch_zero_section(D.U.ref(), c->st);
  D.u_zero = false;
}

// Up sweep and correction of level l (Alg. 1, coarse to fine; Alg. 3 apply
// correction): z = P e_{l-1} (e_{l-1} in the ef array of level l - 1),
// y = S^nu2(y'_l; g_l - A z), y'_l = Q(y), u'_l = Q(dec u'_l + dec y'_l) and,
// below the FMG level, e_l = dec y'_l + z.
template <typename T>
void up_level(cmg_ctx c, int l, int Lp) {
  hipStream_t st = c->st;
  int* nf = c->flags + 1;
  LevelData& F = c->lv[l];
  LevelData& C = c->lv[l - 1];
  const double ih2 = inv_h2(l);
  F.Y.w = c->wy(l, Lp);
  F.Yp.w = c->wy(l, Lp);
  F.U.wt = c->wu(l, Lp);  // the correction writes codes of this width
  if (std::is_same<T, float>::value && c->smooth_fused(l)) {
    const float cp = static_cast<float>(1.0 / (2.0 * c->p.dim * ih2));
    if (!fused_up_smooth(static_cast<const float*>(C.ef), F.G.ref(), F.Y.ref(), F.Yp.ref(), F.U.ref_corr(),
                         l < Lp ? static_cast<float*>(F.ef) : nullptr, F.g, C.g, c->o.nu_post, cp,
                         static_cast<float>(ih2), st, F.u_zero))
      fail(CMG_ERR_HIP, "fused up-smoothing rejected a level it was selected for");
    F.u_zero = false;  // every code of u' is written now, at width wt
    F.U.w = F.U.wt;
    KCK();
    return;
  }
  ensure_u(c, l);
  T* yf = static_cast<T*>(F.yf);
  T* zf = static_cast<T*>(F.zf);
  T* rf = static_cast<T*>(F.rf);
  launch_prolong<T>(static_cast<T*>(C.ef), F.g, C.g, zf, st);
  launch_dec_minus_A<T>(F.G.ref(), zf, kapT<T>(c, l), F.g, static_cast<T>(ih2), rf, st);  // dec g - A z
  smooth_from_section<T>(c, l, F.Y.ref(), yf, rf, static_cast<T*>(F.ef), c->o.nu_post);
  // y' = Q(y); u' = Q(dec u' + dec y'); below the top level e_l = dec y' + z
  const SecRef u = F.U.ref_corr();
  launch_encode_dec<T>(yf, F.g.size, F.Yp.ref(), nf, l < Lp ? static_cast<T*>(F.ef) : nullptr, zf, &u, st);
  F.U.w = F.U.wt;
  KCK();
}

// One compact V-cycle from zero on G[Lp], then u' += y' (Alg. 1, Alg. 3).
// Levels with rows of >= 64 nodes run the fused 3-D kernels; the others (and
// every 2-D, Jacobi or diffusion level) run one kernel per operation.
template <typename T>
void vcycle_correct(cmg_ctx c, int Lp) {
  const int lc = c->lc();
  hipStream_t st = c->st;
  int* nf = c->flags + 1;
  constexpr bool f32 = std::is_same<T, float>::value;
  // Lc: the top of the small levels that one workgroup cycles through
  int Lc = lc;
  for (int l = std::min(Lp, kCoarseMaxLevel); l > lc; --l)
    if (coarse_pool_bytes(c->p.dim, lc, l, sizeof(T)) <= kCoarsePoolBytes && !c->smooth_fused(l) &&
        c->lv[lc].g.size <= kCoarsestMax) {
      Lc = l;
      break;
    }
  for (int l = Lp; l > Lc; --l) {  // fine to coarse
    LevelData& F = c->lv[l];
    LevelData& C = c->lv[l - 1];
    const double ih2 = inv_h2(l);
    F.Y.w = c->wy(l, Lp);
    if (c->chain()) {  // V(0, nu2): y' = Q(0), s = 0; g_{l-1} = r_{l-1} came from the IR residual
      launch_zero_section(F.Y.ref(), st);
      KCK();
      continue;
    }
    C.G.w = c->wr(l - 1, Lp);
    const bool fs = f32 && c->smooth_fused(l);
    if (fs && c->o.nu_pre == 0) {  // V(0, nu2): y' = Q(0)
      launch_zero_section(F.Y.ref(), st);
      KCK();
    } else if (fs) {
      const float cp = static_cast<float>(1.0 / (2.0 * c->p.dim * ih2));
      if (!fused_down_smooth(F.G.ref(), F.Y.ref(), F.g, c->o.nu_pre, cp, static_cast<float>(ih2), st))
        fail(CMG_ERR_HIP, "fused down-smoothing rejected a level it was selected for");
      KCK();
    }
    if (f32 && c->rr_fused(l)) {
      if (!fused_resid_restrict(F.G.ref(), F.Y.ref(), C.G.ref(), F.g, C.g, static_cast<float>(ih2), st))
        fail(CMG_ERR_HIP, "fused residual restriction rejected a level it was selected for");
      KCK();
      continue;
    }
    T* gf = static_cast<T*>(F.gf);
    T* yf = static_cast<T*>(F.yf);
    T* rf = static_cast<T*>(F.rf);
    launch_decode<T>(F.G.ref(), F.g.size, gf, st);
    if (!fs) {
      smooth_from_zero<T>(c, l, yf, gf, static_cast<T*>(F.ef), c->o.nu_pre);
      launch_encode_dec<T>(yf, F.g.size, F.Y.ref(), nf, yf, nullptr, nullptr, st);  // y' = Q(y); yf = dec y'
    } else {
      launch_decode<T>(F.Y.ref(), F.g.size, yf, st);
    }
    launch_rhs_minus_A<T>(gf, yf, kapT<T>(c, l), F.g, static_cast<T>(ih2), rf, st);
    launch_restrict_encode<T>(rf, C.g, F.g, C.G.ref(), nf, st);  // g_{l-1} = Q(R(g - A y'))
    KCK();
  }
  LevelData& B = c->lv[lc];  // coarsest, float64
  if (Lc > lc) {  // levels lc .. Lc in one workgroup
    CoarseArgs a{};
    for (int l = lc; l <= Lc; ++l) {
      LevelData& D = c->lv[l];
      D.Y.w = c->wy(l, Lp);
      D.Yp.w = c->wy(l, Lp);
      D.U.wt = c->wu(l, Lp);
      if (l < Lc) D.G.w = c->wr(l, Lp);
      CoarseLevel& q = a.lv[l];
      q.G = D.G.ref();
      q.Y = D.Y.ref();
      q.Yp = D.Yp.ref();
      q.U = D.U.ref_corr();
      q.ef = D.ef;
      a.off[l] = l == lc ? 0 : a.off[l - 1] + 5 * static_cast<int>(c->lv[l - 1].g.size);
      q.kap = kapT<T>(c, l);
      q.g = D.g;
      q.ih2 = inv_h2(l);
      q.cp = (c->o.smoother == CMG_RBGS ? 1.0 : c->o.omega) / (2.0 * c->p.dim * q.ih2);
    }
    a.kap64 = kap64(c, lc);
    a.lc = lc;
    a.Lc = Lc;
    a.Lp = Lp;
    a.nu_pre = c->o.nu_pre;
    a.nu_post = c->o.nu_post;
    a.rbgs = c->o.smoother == CMG_RBGS ? 1 : 0;
    a.omega = c->o.omega;
    a.chain = c->chain() ? 1 : 0;
    a.nonfinite = nf;
    launch_coarse_vcycle<T>(a, st);
    for (int l = lc; l <= Lc; ++l) c->lv[l].U.w = c->lv[l].U.wt;  // corrected at width wt
    KCK();
  } else {
    launch_decode<double>(B.G.ref(), B.g.size, B.t64, st);
    launch_coarse_single(B.t64, kap64(c, lc), B.g, inv_h2(lc), B.s64, st);
    B.Yp.w = c->wy(lc, Lp);
    launch_encode<double>(B.s64, B.g.size, B.Yp.ref(), nf, st);
    B.U.wt = c->wu(lc, Lp);
    launch_correct(B.U.ref_corr(), B.Yp.ref(), st);
    B.U.w = B.U.wt;
    launch_decode<T>(B.Yp.ref(), B.g.size, static_cast<T*>(B.ef), st);
    KCK();
  }
  for (int l = Lc + 1; l <= Lp; ++l) up_level<T>(c, l, Lp);  // coarse to fine
}

// Decoded solution u_l = dec u'_l + P u_{l-1} for levels lc .. top (float64).
void decode_chain(cmg_ctx c, int top) {
  const int lc = c->lc();
  for (int l = lc; l <= top; ++l) ensure_u(c, l);
  launch_decode<double>(c->lv[lc].U.ref(), c->lv[lc].g.size, c->lv[lc].uh, c->st);
  for (int l = lc + 1; l <= top; ++l)
    if (!fused_decode_level(c->lv[l].U.ref(), c->lv[l - 1].uh, c->lv[l].g, c->lv[l - 1].g, c->lv[l].uh, c->st))
      launch_prolong_add_dec(c->lv[l].U.ref(), c->lv[l - 1].uh, c->lv[l].g, c->lv[l - 1].g, c->lv[l].uh, c->st);
  KCK();
}

// Decoded solution of FMG level Lp into a full node array (Lp + 1)^dim.
// Where u_{Lp-1} is not stored (skip_fused), `spare` (a section whose codes
// are dead, e.g. y' of the finest level at the end of a solve) may hold it:
// it is decoded there in one pass and the final decode reads it; otherwise
// the final decode rebuilds it plane by plane.
void decode_to_full(cmg_ctx c, int Lp, double* u, const Section* spare = nullptr) {
  ensure_u(c, Lp);
  if (c->p.dim == 3 && Lp > c->lc() && c->lv[Lp].g.n >= 64) {
    const bool skip = c->skip_fused(Lp);
    decode_chain(c, skip ? Lp - 2 : Lp - 1);
    LevelData& C = c->lv[Lp - 1];
    double* uc = skip ? nullptr : C.uh;
    if (skip && spare != nullptr && spare->bytes >= 8 * C.g.size) {
      uc = static_cast<double*>(spare->codes);
      if (!fused_decode_level(C.U.ref(), c->lv[Lp - 2].uh, C.g, c->lv[Lp - 2].g, uc, c->st))
        launch_prolong_add_dec(C.U.ref(), c->lv[Lp - 2].uh, C.g, c->lv[Lp - 2].g, uc, c->st);
    }
    const bool rebuild = uc == nullptr;
    const SecRef ucs = C.U.ref();
    if (!fused_decode_full(c->lv[Lp].U.ref(), uc, c->lv[Lp].g, C.g, u, c->st, rebuild ? &ucs : nullptr,
                           rebuild ? c->lv[Lp - 2].uh : nullptr))
      fail(CMG_ERR_HIP, "fused decode rejected a level it was selected for");
  } else {
    decode_chain(c, Lp);
    launch_to_full(c->lv[Lp].uh, c->lv[Lp].g, u, c->st);
  }
  KCK();
}

// Alg. 2, "restrict residual": t_{l-1} = R t_l in float64 from the
// unrounded t64[top], every level rounded once into its residual section
// (levels top - 1 .. lc).
void residual_chain(cmg_ctx c, int Lp, int top) {
  for (int l = top - 1; l >= c->lc(); --l) {
    LevelData& D = c->lv[l];
    launch_restrict<double>(c->lv[l + 1].t64, D.g, c->lv[l + 1].g, D.t64, c->st);
    D.G.w = c->wr(l, Lp);
    launch_encode<double>(D.t64, D.g.size, D.G.ref(), c->flags + 1, c->st);
  }
  KCK();
}

// IR residual (Alg. 2) into G[Lp] (and, for a cycle without pre-smoothing,
// into every coarser G).  f is the caller's finest node array; the
// per-operation path uses the injected copy in f64[Lp].  Every residual also
// feeds the divergence monitor: its sum of squares is compared with the
// smallest one of the same FMG level (k_monitor_check).
constexpr double kDivergeGrowth = 4.0;  // residual norm growth that counts as divergence

void ir_residual(cmg_ctx c, int Lp, const double* f, cmg_stats* st, bool watch = true) {
  LevelData& F = c->lv[Lp];
  F.G.w = c->wr(Lp, Lp);
  const bool rec = st != nullptr && st->record && st->count < 256;
  launch_monitor_reset(c->mon, c->mon_fresh, c->st);
  c->mon_fresh = false;
  if (c->res_fused(Lp)) {
    const bool skip = c->skip_fused(Lp);
    decode_chain(c, skip ? Lp - 2 : Lp - 1);
    const SecRef uc = c->lv[Lp - 1].U.ref();
    if (!fused_ir_residual(F.U.ref(), skip ? nullptr : c->lv[Lp - 1].uh, f, c->p.L, F.g, c->lv[Lp - 1].g, inv_h2(Lp),
                           F.G.ref(), c->flags + 1, c->mon, c->st, skip ? &uc : nullptr,
                           skip ? c->lv[Lp - 2].uh : nullptr, F.u_zero))
      fail(CMG_ERR_HIP, "fused IR residual rejected a level it was selected for");
    KCK();
  } else {
    decode_chain(c, Lp);
    if (!c->chain()) {  // residual and encode in one pass
      launch_res_encode(F.f64, F.uh, kap64(c, Lp), F.g, inv_h2(Lp), F.G.ref(), c->flags + 1, c->mon, c->st);
      KCK();
    } else {  // the restriction chain needs the residual array
      launch_rhs_minus_A<double>(F.f64, F.uh, kap64(c, Lp), F.g, inv_h2(Lp), F.t64, c->st);
      launch_encode<double>(F.t64, F.g.size, F.G.ref(), c->flags + 1, c->st);
      launch_sumsq(F.t64, F.g.size, c->mon, c->st);
      KCK();
      residual_chain(c, Lp, Lp);
    }
  }
  if (watch) launch_monitor_check(c->mon, c->flags, Lp, kDivergeGrowth, c->st);
  KCK();
  if (rec) {
    double h = 0.0;
    HIPCK(hipMemcpyAsync(&h, c->mon + kMonLast, 8, hipMemcpyDeviceToHost, c->st));
    HIPCK(hipStreamSynchronize(c->st));
    st->residual_norm[st->count++] = std::sqrt(h);
  }
}

void enter_level(cmg_ctx c, int level, const double* f) {
  const int lc = c->lc();
  LevelData& D = c->lv[level];
  if (level == lc) {
    launch_inject(f, c->p.L, D.g, D.f64, c->st);
    launch_coarse_single(D.f64, kap64(c, lc), D.g, inv_h2(lc), D.s64, c->st);
    D.U.set_w(c->wu(lc, lc));
    launch_encode<double>(D.s64, D.g.size, D.U.ref(), c->flags + 1, c->st);
    D.u_zero = false;
    KCK();
  } else {
    // the coarser u' sections take the new level's widths (Table 1) at their
    // first correction on it: widening only appends zero bits to the codes
    for (int l = lc; l < level; ++l) {
      ensure_u(c, l);
      c->lv[l].U.wt = c->wu(l, level);
    }
    D.U.set_w(c->wu(level, level));
    if (c->u_lazy(level)) {
      D.u_zero = true;
    } else {
      D.u_zero = false;
      launch_zero_section(D.U.ref(), c->st);
    }
    if (D.f64 != nullptr) launch_inject(f, c->p.L, D.g, D.f64, c->st);
    KCK();
  }
  c->Lp = level;
  c->mon_fresh = true;
}

template <typename T>
void compact_fmg_one(cmg_ctx c, const double* f, double* u, cmg_stats* st) {
  const int L = c->p.L;
  for (int level = c->lc(); level <= L; ++level) {
    enter_level(c, level, f);
    if (level == c->lc()) continue;
    const int iters = c->o.ir_iters + (level == L ? c->o.final_iters : 0);
    for (int it = 0; it < iters; ++it) {
      ir_residual(c, level, f, st);
      vcycle_correct<T>(c, level);
    }
  }
  // y' of the finest level is dead now (and not exported without
  // keep_correction): its buffer holds u_{L-1} for the final decode
  decode_to_full(c, L, u, c->o.keep_correction ? nullptr : &c->lv[L].Y);
}

// Correction-scheme V(nu1, nu2) cycle (supplement Sec. SM1.1.1) on rf[Lp];
// result in yf[Lp].  In place on the level arrays r and y: red-black sweeps
// one half-sweep per launch, the restriction of the residual and the
// prolongation-add each in one kernel (weighted Jacobi alternates with zf).
template <typename T>
void cs_vcycle(cmg_ctx c, int Lp) {
  const int lc = c->lc();
  hipStream_t st = c->st;
  for (int l = Lp; l > lc; --l) {
    LevelData& F = c->lv[l];
    LevelData& C = c->lv[l - 1];
    T* yf = static_cast<T*>(F.yf);
    T* rf = static_cast<T*>(F.rf);
    smooth_from_zero<T>(c, l, yf, rf, static_cast<T*>(F.zf), c->o.nu_pre);
    if (F.zf != nullptr) {  // residual into the free sweep scratch, then restricted: two coalesced passes
      launch_rhs_minus_A<T>(rf, yf, kapT<T>(c, l), F.g, static_cast<T>(inv_h2(l)), static_cast<T*>(F.zf), st);
      launch_restrict<T>(static_cast<const T*>(F.zf), C.g, F.g, static_cast<T*>(C.rf), st);
    } else {
      launch_restrict_residual<T>(rf, yf, kapT<T>(c, l), C.g, F.g, static_cast<T>(inv_h2(l)), static_cast<T*>(C.rf),
                                  st);
    }
    KCK();
  }
  LevelData& B = c->lv[lc];
  launch_convert<T, double>(static_cast<T*>(B.rf), B.t64, B.g.size, st);
  launch_coarse_single(B.t64, kap64(c, lc), B.g, inv_h2(lc), B.s64, st);
  launch_convert<double, T>(B.s64, static_cast<T*>(B.yf), B.g.size, st);
  KCK();
  for (int l = lc + 1; l <= Lp; ++l) {
    LevelData& F = c->lv[l];
    LevelData& C = c->lv[l - 1];
    T* yf = static_cast<T*>(F.yf);
    launch_prolong_add<T>(static_cast<T*>(C.yf), F.g, C.g, yf, st);
    KCK();
    smooth<T>(c, l, yf, static_cast<T*>(F.rf), static_cast<T*>(F.zf), c->o.nu_post);
  }
}

// Plain FMG (Alg. SM2) on float64 standard vectors: the solution of FMG
// level l lives in pu[(L - l) & 1], so that the prolongation to the next
// level reads one buffer and writes the other.
template <typename T>
void plain_fmg_one(cmg_ctx c, const double* f, double* u, cmg_stats* st) {
  const int L = c->p.L, lc = c->lc();
  hipStream_t s = c->st;
  auto ubuf = [&](int level) { return c->pu[(L - level) & 1]; };
  LevelData& B = c->lv[lc];
  launch_inject(f, L, B.g, B.f64, s);
  launch_coarse_single(B.f64, kap64(c, lc), B.g, inv_h2(lc), ubuf(lc), s);
  KCK();
  for (int level = lc + 1; level <= L; ++level) {
    LevelData& F = c->lv[level];
    launch_prolong<double>(ubuf(level - 1), F.g, c->lv[level - 1].g, ubuf(level), s);
    KCK();
    const int iters = c->o.ir_iters + (level == L ? c->o.final_iters : 0);
    for (int it = 0; it < iters; ++it) {
      launch_monitor_reset(c->mon, it == 0, s);
      launch_residual_full<T>(f, L, ubuf(level), kap64(c, level), F.g, inv_h2(level), static_cast<T*>(F.rf),
                              c->flags + 1, c->mon, s);
      launch_monitor_check(c->mon, c->flags, level, kDivergeGrowth, s);
      KCK();
      if (st != nullptr && st->record && st->count < 256) {
        double h = 0.0;
        HIPCK(hipMemcpyAsync(&h, c->mon + kMonLast, 8, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        st->residual_norm[st->count++] = std::sqrt(h);
      }
      cs_vcycle<T>(c, level);
      launch_add_correction<T>(ubuf(level), static_cast<T*>(F.yf), F.g.size, s);
      KCK();
    }
  }
  launch_to_full(ubuf(L), c->lv[L].g, u, s);
  KCK();
}

void fmg_one(cmg_ctx c, const double* f, double* u, cmg_stats* st) {
  const bool f32 = c->o.vcycle_prec == CMG_FP32;
  if (c->compact()) {
    if (f32) compact_fmg_one<float>(c, f, u, st);
    else compact_fmg_one<double>(c, f, u, st);
  } else {
    if (f32) plain_fmg_one<float>(c, f, u, st);
    else plain_fmg_one<double>(c, f, u, st);
  }
}

void check_flags(cmg_ctx c) {
  int h[3] = {0, 0, 0};
  HIPCK(hipMemcpyAsync(h, c->flags, sizeof(h), hipMemcpyDeviceToHost, c->st));
  HIPCK(hipStreamSynchronize(c->st));
  if (h[1] || h[2]) HIPCK(hipMemsetAsync(c->flags, 0, sizeof(h), c->st));
  if (h[1]) fail(CMG_ERR_NONFINITE, "non-finite value met during the solve (NaN/Inf in the input?)");
  if (h[2])
    fail(CMG_ERR_NOT_CONVERGED, "the IR residual grew to more than " + std::to_string(kDivergeGrowth) +
                                    " times its smallest norm on FMG level " + std::to_string(h[2]) +
                                    ": the iteration diverges (smoother, widths or coefficients)");
}

// Installs the context's timing sink for the duration of one API call and
// folds the recorded events into the totals when the call ends.
struct TimingScope {
  cmg_ctx c;
  explicit TimingScope(cmg_ctx ctx) : c(ctx) { g_timing = (c != nullptr && c->timing_on) ? &c->timing : nullptr; }
  ~TimingScope() {
    if (g_timing != nullptr) g_timing->flush();
    g_timing = nullptr;
  }
};

template <typename Fn>
cmg_status guard(cmg_ctx c, Fn&& fn) {
  try {
    if (c != nullptr && c->dead) fail(CMG_ERR_INVALID_ARG, "context unusable after an earlier HIP failure");
    TimingScope ts(c);
    fn();
    return CMG_OK;
  } catch (const CmgError& e) {
    if (c != nullptr) {
      c->err = e.msg;
      if (e.code == CMG_ERR_HIP || e.code == CMG_ERR_OUT_OF_MEMORY) c->dead = true;
    } else {
      g_thread_error = e.msg;
    }
    return e.code;
  } catch (const std::exception& e) {
    if (c != nullptr) c->err = e.what(); else g_thread_error = e.what();
    return CMG_ERR_HIP;
  } catch (...) {
    if (c != nullptr) c->err = "unknown error"; else g_thread_error = "unknown error";
    return CMG_ERR_HIP;
  }
}

void need(bool ok, const char* msg) {
  if (!ok) fail(CMG_ERR_INVALID_ARG, msg);
}

Section& section_of(cmg_ctx c, int which, int level) {
  if (!c->compact()) fail(CMG_ERR_UNSUPPORTED, "plain storage has no compact sections");
  need(level >= c->lc() && level <= c->p.L, "level out of range");
  LevelData& D = c->lv[level];
  if (which == CMG_SECTION_U) return D.U;
  if (which == CMG_SECTION_R) return D.G;
  if ((which == CMG_SECTION_Y || which == CMG_SECTION_YPRE) && !c->o.keep_correction)
    fail(CMG_ERR_UNSUPPORTED, "the correction sections are kept only in contexts set up with keep_correction = 1");
  if (which == CMG_SECTION_Y) return D.Yp;
  if (which == CMG_SECTION_YPRE) return D.Y;
  fail(CMG_ERR_INVALID_ARG, "unknown section kind");
}

void release(cmg_ctx c) {
  (void)hipStreamSynchronize(c->st);
  for (void* ptr : c->allocs) (void)hipFree(ptr);
  c->allocs.clear();
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

cmg_status cmg_default_opts(cmg_opts* o) {
  if (o == nullptr) {
    g_thread_error = "options must not be NULL";
    return CMG_ERR_INVALID_ARG;
  }
  std::memset(o, 0, sizeof(*o));
  o->smoother = CMG_RBGS;
  o->omega = 0.8;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->ir_iters = 2;
  o->vcycles = 1;
  o->final_iters = 0;
  o->storage = CMG_COMPACT_BFP;
  o->bfp_block = 64;
  o->bits_u = o->bits_r = o->bits_y = 16;
  o->inc_u = 2;
  o->inc_ry = 1;
  o->vcycle_prec = CMG_FP32;
  return CMG_OK;
}

cmg_status cmg_setup(const cmg_problem* p, const cmg_opts* o, const double* kappa_cells, void* hip_stream,
                     cmg_ctx* out) {
  if (out == nullptr) {
    g_thread_error = "out must not be NULL";
    return CMG_ERR_INVALID_ARG;
  }
  *out = nullptr;
  cmg_status s = guard(nullptr, [&] {
    validate(p, o);
    if (p->op == CMG_DIFFUSION && kappa_cells == nullptr) fail(CMG_ERR_INVALID_ARG, "diffusion needs kappa");
  });
  if (s != CMG_OK) return s;
  cmg_ctx c = new (std::nothrow) cmg_ctx_s();
  if (c == nullptr) {
    g_thread_error = "host allocation failed";
    return CMG_ERR_OUT_OF_MEMORY;
  }
  c->p = *p;
  c->o = *o;
  c->st = static_cast<hipStream_t>(hip_stream);
  s = guard(c, [&] { setup_levels(c, kappa_cells); });
  if (s != CMG_OK) {
    g_thread_error = c->err;
    try {
      release(c);
    } catch (...) {
    }
    delete c;
    return s;
  }
  *out = c;
  return CMG_OK;
}

cmg_status cmg_fmg_solve(cmg_ctx c, const double* f, double* u, cmg_stats* st) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(f != nullptr && u != nullptr, "f and u must not be NULL");
    if (st != nullptr) st->count = 0;
    const int64_t M = c->full_size(c->p.L);
    for (int b = 0; b < c->p.batch; ++b) fmg_one(c, f + b * M, u + b * M, st);
    check_flags(c);
  });
}

cmg_status cmg_vcycle(cmg_ctx c, const double* r, double* y) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(r != nullptr && y != nullptr, "r and y must not be NULL");
    const int L = c->p.L, lc = c->lc();
    const int64_t M = c->full_size(L);
    const bool f32 = c->o.vcycle_prec == CMG_FP32;
    for (int b = 0; b < c->p.batch; ++b) {
      LevelData& F = c->lv[L];
      if (c->compact()) {
        F.G.w = c->wr(L, L);  // r rounded to the finest residual width
        if (c->chain()) {  // and restricted unrounded to every level (Alg. 2)
          launch_inject(r + b * M, L, F.g, F.t64, c->st);
          launch_encode<double>(F.t64, F.g.size, F.G.ref(), c->flags + 1, c->st);
          KCK();
          residual_chain(c, L, L);
        } else {
          launch_encode_full(r + b * M, L, F.g, F.G.ref(), c->flags + 1, c->st);
        }
        for (int l = lc; l <= L; ++l) {
          c->lv[l].U.set_w(c->wu(l, L));
          launch_zero_section(c->lv[l].U.ref(), c->st);
          c->lv[l].u_zero = false;
        }
        KCK();
        c->Lp = L;
        if (f32) vcycle_correct<float>(c, L); else vcycle_correct<double>(c, L);
        decode_to_full(c, L, y + b * M);
      } else {  // r - A 0 = r sampled into the level array, then y from zero
        double* u0 = c->pu[0];
        launch_fill<double>(u0, 0.0, F.g.size, c->st);
        launch_monitor_reset(c->mon, true, c->st);
        if (f32) {
          launch_residual_full<float>(r + b * M, L, u0, nullptr, F.g, inv_h2(L), static_cast<float*>(F.rf),
                                      c->flags + 1, c->mon, c->st);
          cs_vcycle<float>(c, L);
          launch_add_correction<float>(u0, static_cast<float*>(F.yf), F.g.size, c->st);
        } else {
          launch_residual_full<double>(r + b * M, L, u0, nullptr, F.g, inv_h2(L), static_cast<double*>(F.rf),
                                       c->flags + 1, c->mon, c->st);
          cs_vcycle<double>(c, L);
          launch_add_correction<double>(u0, static_cast<double*>(F.yf), F.g.size, c->st);
        }
        launch_to_full(u0, F.g, y + b * M, c->st);
      }
      KCK();
    }
    check_flags(c);
  });
}

cmg_status cmg_adjoint_solve(cmg_ctx c, const double* u, const double* dJdu, double* lambda, double* grad_kappa) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(u != nullptr && dJdu != nullptr && lambda != nullptr, "u, dJdu and lambda must not be NULL");
    if (grad_kappa != nullptr && c->p.op != CMG_DIFFUSION)
      fail(CMG_ERR_INVALID_ARG, "grad_kappa needs the diffusion operator");
    const int64_t M = c->full_size(c->p.L);
    const Geom gcell = make_geom(c->p.dim, c->p.L);
    for (int b = 0; b < c->p.batch; ++b) {
      fmg_one(c, dJdu + b * M, lambda + b * M, nullptr);
      if (grad_kappa != nullptr) {
        launch_grad_kappa(u + b * M, lambda + b * M, gcell, b > 0 ? 1 : 0, grad_kappa, c->st);
        KCK();
      }
    }
    check_flags(c);
  });
}

cmg_status cmg_destroy(cmg_ctx c) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  try {
    release(c);
  } catch (...) {
  }
  delete c;
  return CMG_OK;
}

const char* cmg_last_error(cmg_ctx c) { return c != nullptr ? c->err.c_str() : g_thread_error.c_str(); }

int64_t cmg_bfp_code_bytes(int64_t n, int32_t block, int32_t bits) {
  if (n < 0 || (block != 32 && block != 64) || bits < 2 || bits > 53) return -1;
  return code_bytes(n, block, bits);
}

cmg_status cmg_bfp_encode(const void* x, int32_t x_is_f64, int64_t n, int32_t block, int32_t bits, void* codes,
                          int16_t* exps, void* hip_stream) {
  return guard(nullptr, [&] {
    need(n >= 0 && (block == 32 || block == 64) && bits >= 2 && bits <= 53, "bad size, block or bits");
    need(n == 0 || (x != nullptr && codes != nullptr && exps != nullptr), "NULL buffer");
    if (n == 0) return;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    SecRef s{codes, exps, n, block, bits, container_bits(bits)};
    // the non-finite flag comes from the stream-ordered pool (no device-wide
    // synchronisation, unlike hipMalloc / hipFree)
    int* flag = nullptr;
    HIPCK(hipMallocAsync(reinterpret_cast<void**>(&flag), sizeof(int), st));
    int h = 0;
    try {
      HIPCK(hipMemsetAsync(flag, 0, sizeof(int), st));
      if (x_is_f64) launch_encode<double>(static_cast<const double*>(x), n, s, flag, st);
      else launch_encode<float>(static_cast<const float*>(x), n, s, flag, st);
      KCK();
      HIPCK(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    } catch (...) {
      (void)hipFreeAsync(flag, st);
      throw;
    }
    HIPCK(hipFreeAsync(flag, st));
    HIPCK(hipStreamSynchronize(st));
    if (h) fail(CMG_ERR_NONFINITE, "codec input holds NaN or Inf");
  });
}

cmg_status cmg_bfp_decode(const void* codes, const int16_t* exps, int64_t n, int32_t block, int32_t bits, double* x,
                          void* hip_stream) {
  return guard(nullptr, [&] {
    need(n >= 0 && (block == 32 || block == 64) && bits >= 2 && bits <= 53, "bad size, block or bits");
    need(n == 0 || (x != nullptr && codes != nullptr && exps != nullptr), "NULL buffer");
    if (n == 0) return;
    SecRef s{const_cast<void*>(codes), const_cast<int16_t*>(exps), n, block, bits, container_bits(bits)};
    launch_decode<double>(s, n, x, static_cast<hipStream_t>(hip_stream));
    KCK();
  });
}

int64_t cmg_abfp_code_bytes(int64_t n, int32_t bits) {
  if (n < 0 || bits < 2 || bits > 53) return -1;
  return code_bytes(n, 64, bits);
}

int64_t cmg_abfp_workspace_bytes(int64_t n) { return n < 0 ? -1 : abfp_workspace_bytes(n); }

cmg_status cmg_abfp_encode(const void* x, int32_t x_is_f64, int64_t n, int32_t bits, void* codes, int64_t* starts,
                           int16_t* exps, int32_t* nblocks, void* workspace, void* hip_stream) {
  return guard(nullptr, [&] {
    need(n >= 0 && bits >= 2 && bits <= 53, "bad size or bits");
    need(n <= (int64_t{1} << 43), "n too large for the tile ticket");
    need(starts != nullptr && exps != nullptr && nblocks != nullptr && workspace != nullptr, "NULL buffer");
    need(n == 0 || (x != nullptr && codes != nullptr), "NULL buffer");
    need(reinterpret_cast<uintptr_t>(codes) % 16 == 0 && reinterpret_cast<uintptr_t>(workspace) % 8 == 0,
         "codes must be 16-byte and workspace 8-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int cb = container_bits(bits);
    if (x_is_f64)
      launch_abfp_encode<double>(static_cast<const double*>(x), n, bits, cb, codes, starts, exps, nblocks, workspace,
                                 st);
    else
      launch_abfp_encode<float>(static_cast<const float*>(x), n, bits, cb, codes, starts, exps, nblocks, workspace,
                                st);
    KCK();
  });
}

cmg_status cmg_abfp_encode_noalloc(const void* x, int32_t x_is_f64, int64_t n, int32_t bits, void* codes,
                                   int64_t* starts, int16_t* exps, int32_t* nblocks, void* hip_stream) {
  return guard(nullptr, [&] {
    need(n >= 0 && n <= kAbNoAllocMax, "n must lie in [0, 2^31]: the static workspace holds no more");
    need(bits >= 2 && bits <= 53, "bad bits");
    need(starts != nullptr && exps != nullptr && nblocks != nullptr, "NULL buffer");
    need(n == 0 || (x != nullptr && codes != nullptr), "NULL buffer");
    need(reinterpret_cast<uintptr_t>(codes) % 16 == 0, "codes must be 16-byte aligned");
    void* ws = abfp_static_workspace();
    if (ws == nullptr) fail(CMG_ERR_HIP, "hipGetSymbolAddress gave no address for the static workspace");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int cb = container_bits(bits);
    if (x_is_f64)
      launch_abfp_encode<double>(static_cast<const double*>(x), n, bits, cb, codes, starts, exps, nblocks, ws, st);
    else
      launch_abfp_encode<float>(static_cast<const float*>(x), n, bits, cb, codes, starts, exps, nblocks, ws, st);
    KCK();
  });
}

cmg_status cmg_abfp_decode(const void* codes, const int64_t* starts, const int16_t* exps, const int32_t* nblocks,
                           int64_t n, int32_t bits, double* x, void* hip_stream) {
  return guard(nullptr, [&] {
    need(n >= 0 && bits >= 2 && bits <= 53, "bad size or bits");
    need(starts != nullptr && exps != nullptr && nblocks != nullptr, "NULL buffer");
    need(n == 0 || (x != nullptr && codes != nullptr), "NULL buffer");
    need(reinterpret_cast<uintptr_t>(codes) % 16 == 0, "codes must be 16-byte aligned");
    if (n == 0) return;
    launch_abfp_decode(codes, starts, exps, nblocks, n, bits, container_bits(bits), x,
                       static_cast<hipStream_t>(hip_stream));
    KCK();
  });
}

cmg_status cmg_section_info(cmg_ctx c, int32_t which, int32_t level, int64_t* n_values, int32_t* bits,
                            int32_t* cbits, int64_t* bytes, int64_t* nblk) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    Section& s = section_of(c, which, level);
    if (n_values) *n_values = s.n;
    if (bits) *bits = which == CMG_SECTION_U && s.wt > s.w ? s.wt : s.w;  // u': its width on this FMG level
    if (cbits) *cbits = s.cbits;
    if (bytes) *bytes = s.bytes;
    if (nblk) *nblk = s.nblk;
  });
}

cmg_status cmg_export_section(cmg_ctx c, int32_t which, int32_t level, void* codes_host, int16_t* exps_host) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    Section& s = section_of(c, which, level);
    need(codes_host != nullptr && exps_host != nullptr, "NULL buffer");
    if (which == CMG_SECTION_U) {
      ensure_u(c, level);
      if (s.wt > s.w) {  // codes of the section's width on this FMG level
        launch_widen(s.ref(), s.wt - s.w, c->st);
        s.w = s.wt;
      }
    }
    HIPCK(hipMemcpyAsync(codes_host, s.codes, static_cast<size_t>(s.bytes), hipMemcpyDeviceToHost, c->st));
    HIPCK(hipMemcpyAsync(exps_host, s.exps, static_cast<size_t>(s.nblk) * 2, hipMemcpyDeviceToHost, c->st));
    HIPCK(hipStreamSynchronize(c->st));
  });
}

cmg_status cmg_import_section(cmg_ctx c, int32_t which, int32_t level, int32_t bits, const void* codes_host,
                              const int16_t* exps_host) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    Section& s = section_of(c, which, level);
    need(codes_host != nullptr && exps_host != nullptr, "NULL buffer");
    need(bits >= 2 && container_bits(bits) <= s.cbits && bits <= 53, "bits do not fit the section's container");
    need(container_bits(bits) == s.cbits || s.cbits != 12, "12-bit container needs 9..12 bits");
    HIPCK(hipMemcpyAsync(s.codes, codes_host, static_cast<size_t>(s.bytes), hipMemcpyHostToDevice, c->st));
    HIPCK(hipMemcpyAsync(s.exps, exps_host, static_cast<size_t>(s.nblk) * 2, hipMemcpyHostToDevice, c->st));
    HIPCK(hipStreamSynchronize(c->st));
    s.set_w(bits);
    if (which == CMG_SECTION_U) c->lv[level].u_zero = false;
  });
}

cmg_status cmg_fmg_enter_level(cmg_ctx c, int32_t level, const double* f) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    if (!c->compact()) fail(CMG_ERR_UNSUPPORTED, "stepwise driving needs compact storage");
    need(f != nullptr, "f must not be NULL");
    need(level == c->lc() || (level == c->Lp + 1 && level <= c->p.L),
         "levels are entered in order, starting at the coarsest");
    enter_level(c, level, f);
  });
}

cmg_status cmg_ir_residual(cmg_ctx c, const double* f) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(f != nullptr, "f must not be NULL");
    need(c->Lp > c->lc(), "enter an FMG level above the coarsest first");
    if (c->lv[c->Lp].f64 != nullptr) launch_inject(f, c->p.L, c->lv[c->Lp].g, c->lv[c->Lp].f64, c->st);
    KCK();
    ir_residual(c, c->Lp, f, nullptr, false);  // stepwise: not watched for divergence
  });
}

cmg_status cmg_vcycle_correct(cmg_ctx c) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(c->Lp > c->lc(), "enter an FMG level above the coarsest first");
    if (c->o.vcycle_prec == CMG_FP32) vcycle_correct<float>(c, c->Lp);
    else vcycle_correct<double>(c, c->Lp);
  });
}

cmg_status cmg_up_sweep(cmg_ctx c, int32_t level, const void* e_coarse) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(e_coarse != nullptr, "e_coarse must not be NULL");
    need(c->Lp > c->lc(), "enter an FMG level above the coarsest first");
    need(level > c->lc() && level <= c->Lp, "level must lie in coarsest + 1 .. the current FMG level");
    LevelData& C = c->lv[level - 1];
    const size_t tsz = c->o.vcycle_prec == CMG_FP32 ? 4 : 8;
    need(C.ef != nullptr, "no coarse correction array on that level");
    HIPCK(hipMemcpyAsync(C.ef, e_coarse, static_cast<size_t>(C.g.size) * tsz, hipMemcpyDeviceToDevice, c->st));
    if (c->o.vcycle_prec == CMG_FP32) up_level<float>(c, level, c->Lp);
    else up_level<double>(c, level, c->Lp);
  });
}

cmg_status cmg_decode_solution(cmg_ctx c, double* u) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(u != nullptr, "u must not be NULL");
    need(c->Lp >= c->lc(), "no FMG level entered");
    decode_to_full(c, c->Lp, u);
  });
}

cmg_status cmg_timing_enable(cmg_ctx c, int32_t enable, const char* kernel) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    c->timing.reset();
    c->timing_on = enable != 0;
    c->timing.filter = (kernel != nullptr) ? kernel : "";
  });
}

cmg_status cmg_timing_count(cmg_ctx c, int32_t* count) {
  if (c == nullptr || count == nullptr) return CMG_ERR_INVALID_ARG;
  *count = static_cast<int32_t>(c->timing.names.size());
  return CMG_OK;
}

cmg_status cmg_timing_entry(cmg_ctx c, int32_t index, char* name, int32_t name_len, int64_t* launches,
                            double* total_ms, double* total_bytes) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(index >= 0 && index < static_cast<int32_t>(c->timing.names.size()), "timing index out of range");
    if (name != nullptr && name_len > 0) {
      std::strncpy(name, c->timing.names[index].c_str(), static_cast<size_t>(name_len - 1));
      name[name_len - 1] = 0;
    }
    if (launches) *launches = c->timing.launches[index];
    if (total_ms) *total_ms = c->timing.ms[index];
    if (total_bytes) *total_bytes = c->timing.bytes[index];
  });
}

cmg_status cmg_memory_stats(cmg_ctx c, cmg_mem* out) {
  if (c == nullptr) return CMG_ERR_INVALID_ARG;
  return guard(c, [&] {
    need(out != nullptr, "out must not be NULL");
    std::memset(out, 0, sizeof(*out));
    out->sections = c->mem[kSections];
    out->coarse_fp64 = c->mem[kCoarse64];
    out->coarse_work = c->mem[kCoarseWork];
    out->fine_work = c->mem[kFineWork];
    out->kappa = c->mem[kKappa];
    int64_t total = 0;
    for (int i = 0; i < kNumCat; ++i) total += c->mem[i];
    out->total = total;
    const int L = c->p.L;
    int64_t m = (int64_t{1} << L) - 1;
    out->interior_dofs = c->p.dim == 3 ? m * m * m : m * m;
    double bits = 0.0;
    for (int l = c->lc(); l <= L; ++l) {
      const double n = static_cast<double>(int64_t{1} << (c->p.dim * l));
      if (c->compact()) {
        const double nb = static_cast<double>(n_blocks(static_cast<int64_t>(n), c->o.bfp_block));
        bits += n * (c->wu(l, L) + c->wr(l, L) + c->wy(l, L)) + 3.0 * 16.0 * nb;
      } else {
        bits += 64.0 * n * (l == L ? 3.0 : 2.0);
      }
    }
    out->logical_bits_per_dof = bits / static_cast<double>(out->interior_dofs);
  });
}

}  // extern "C"
