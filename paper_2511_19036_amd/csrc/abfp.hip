// Adaptive-exponent BFP codec (Sec. 6.1.3, Exponents).
//
// The entries of a vector are normalised to the largest exponent seen so
// far; a new block starts wherever that running exponent rises, and only
// the `w` largest exponents (the last `w` blocks) are kept: every other
// block's entries would round to zero at the largest exponent.  On the CPU
// this is one sequential pass; here it is one pass of a decoupled
// look-back scan:
//
//   * a workgroup takes the next tile of 4096 values (a ticket, so that all
//     lower tiles have started), each thread 16 consecutive values;
//   * the per-entry exponents (fixed-block exponent of the entry alone) are
//     scanned with `max` inside the tile, and the tile's maximum is
//     published at once;
//   * wave 0 walks back over the published maxima of the lower tiles, 64
//     at a time, until one that already has its inclusive prefix, and
//     publishes its own;
//   * every entry then knows its running exponent, writes its code, and the
//     entry where the running exponent rises records its index in a table
//     indexed by exponent (each exponent starts at most one block);
//   * a one-thread kernel keeps the `w` largest exponents of that table.
//
// Codes are packed per thread (16 values: 16, 24, 32, 64 or 128 bytes), in
// the containers of the fixed-block codec.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "abfp.h"
#include "plane.h"
#include "timing.h"

namespace cmg {

namespace {

struct AbWork {
  uint32_t ticket;
  uint32_t flags;  // bit 0: non-finite input; bit 1: a look-back gave up
  uint64_t pad;
};

__device__ __forceinline__ int64_t* ab_table(void* w) { return reinterpret_cast<int64_t*>(static_cast<char*>(w) + 16); }
__device__ __forceinline__ uint64_t* ab_status(void* w) {
  return reinterpret_cast<uint64_t*>(static_cast<char*>(w) + 16 + 8 * kAbEtab);
}

constexpr uint64_t kAggregate = 1, kPrefix = 2;  // look-back states (0: not yet published)
constexpr int kSpinLimit = 1 << 22;               // sleeps of 128 cycles before giving up

__device__ __forceinline__ uint64_t pack_state(uint64_t state, int v) {
  return (state << 32) | static_cast<uint32_t>(v);
}

// Codes of 16 consecutive values (first index a multiple of 16) in the
// container of `CB` bits, at byte offset 16 * i0 * CB / 8 of the code buffer.
template <int CB>
__device__ __forceinline__ void store16(char* codes, int64_t i0, const int64_t (&m)[kAbPT]) {
  char* dst = codes + i0 * CB / 8;
  if constexpr (CB == 12) {
    uint32_t wd[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) {
      const uint32_t c = static_cast<uint32_t>(m[k]) & 0xFFFu;
      const int bit = 12 * k, wi = bit >> 5, sh = bit & 31;
      wd[wi] |= c << sh;
      if (sh > 20) wd[wi + 1] |= c >> (32 - sh);
    }
    uint2* d = reinterpret_cast<uint2*>(dst);  // 24 bytes at a multiple of 24: 8-byte aligned
    d[0] = make_uint2(wd[0], wd[1]);
    d[1] = make_uint2(wd[2], wd[3]);
    d[2] = make_uint2(wd[4], wd[5]);
  } else {
    using C = typename std::conditional<CB == 8, int8_t,
              typename std::conditional<CB == 16, int16_t,
              typename std::conditional<CB == 32, int32_t, int64_t>::type>::type>::type;
    C buf[kAbPT];
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) buf[k] = static_cast<C>(m[k]);
    __builtin_memcpy(dst, buf, sizeof(buf));
  }
}

template <int CB>
__device__ __forceinline__ void load16(const char* codes, int64_t i0, int64_t (&m)[kAbPT]) {
  const char* src = codes + i0 * CB / 8;
  if constexpr (CB == 12) {
    uint32_t wd[7];
    __builtin_memcpy(wd, src, 24);
    wd[6] = 0;
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) {
      const int bit = 12 * k, wi = bit >> 5, sh = bit & 31;
      const uint32_t x = __builtin_amdgcn_alignbit(wd[wi + 1], wd[wi], sh);
      m[k] = static_cast<int64_t>(static_cast<int>(x << 20) >> 20);
    }
  } else {
    using C = typename std::conditional<CB == 8, int8_t,
              typename std::conditional<CB == 16, int16_t,
              typename std::conditional<CB == 32, int32_t, int64_t>::type>::type>::type;
    C buf[kAbPT];
    __builtin_memcpy(buf, src, sizeof(buf));
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) m[k] = static_cast<int64_t>(buf[k]);
  }
}

__global__ void k_abfp_prep(void* work, int64_t tiles) {
  const int64_t words = kAbEtab + tiles;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words + 2;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (i < 2) reinterpret_cast<uint64_t*>(work)[i] = 0;                 // ticket, flags, pad
    else if (i < 2 + kAbEtab) ab_table(work)[i - 2] = -1;                  // no block yet
    else ab_status(work)[i - 2 - kAbEtab] = 0;                             // not published
  }
}

template <typename T>
__global__ void __launch_bounds__(kAbNT) k_abfp_encode(const T* __restrict__ x, int64_t n, int w, int cbits,
                                                       char* __restrict__ codes, void* work) {
  __shared__ uint32_t s_tile;
  __shared__ int s_wave[kAbNT / 64];
  __shared__ int s_excl;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  AbWork* hdr = static_cast<AbWork*>(work);
  if (tid == 0) s_tile = atomicAdd(&hdr->ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t i0 = tile * kAbTile + static_cast<int64_t>(kAbPT) * tid;
  const int64_t npad = (n + 63) / 64 * 64;

  // values (0 past n) and their exponents
  double v[kAbPT];
  if (i0 + kAbPT <= n) {
    T buf[kAbPT];
    __builtin_memcpy(buf, x + i0, sizeof(buf));
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) v[k] = static_cast<double>(buf[k]);
  } else {
#pragma unroll
    for (int k = 0; k < kAbPT; ++k) v[k] = i0 + k < n ? static_cast<double>(x[i0 + k]) : 0.0;
  }
  const double lim = exp_lim(0.0, w);
  bool bad = false;
  int run[kAbPT];  // running exponent over this thread's values
  int r = kNoExp;
#pragma unroll
  for (int k = 0; k < kAbPT; ++k) {
    bad = bad || !isfinite(v[k]);
    r = max(r, lane_exp(v[k], lim));
    run[k] = r;
  }
  if (bad) atomicOr(&hdr->flags, 1u);

  // inclusive max-scan of the thread maxima over the tile
  int incl = r;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl = max(incl, t);
  }
  int texcl = __shfl_up(incl, 1, 64);
  if (lane == 0) texcl = kNoExp;
  if (lane == 63) s_wave[wv] = incl;
  __syncthreads();
  int wpre = kNoExp, agg = kNoExp;
#pragma unroll
  for (int q = 0; q < kAbNT / 64; ++q) {
    if (q < wv) wpre = max(wpre, s_wave[q]);
    agg = max(agg, s_wave[q]);
  }
  texcl = max(texcl, wpre);  // running exponent before this thread's values, within the tile

  // Look-back over the lower tiles by wave 0: lane l reads the status word
  // of tile p - l, so 64 predecessors are examined per round; the closest
  // one holding its inclusive prefix ends the walk.  A status word carries
  // its value, so relaxed device-coherent loads and stores suffice.
  if (wv == 0) {
    uint64_t* status = ab_status(work);
    if (lane == 0)
      __hip_atomic_store(&status[tile], pack_state(kAggregate, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int excl = kNoExp;
    int spins = 0;
    for (int64_t p = tile - 1; p >= 0;) {
      const int64_t q = p - lane;
      const uint64_t sw = q >= 0 ? __hip_atomic_load(&status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : pack_state(kPrefix, kNoExp);  // before tile 0: the empty prefix
      const uint64_t state = sw >> 32;
      const uint64_t prefix = __ballot(state == kPrefix), waiting = __ballot(state == 0);
      const int first = prefix ? __ffsll(static_cast<unsigned long long>(prefix)) - 1 : 63;
      const uint64_t upto = first == 63 ? ~0ull : ((2ull << first) - 1);  // lanes 0 .. first
      if (waiting & upto) {  // a closer tile has not published yet
        if (++spins > kSpinLimit) {  // never expected: every tile publishes without waiting
          if (lane == 0) atomicOr(&hdr->flags, 2u);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
        continue;
      }
      const int val = lane <= first ? static_cast<int>(static_cast<uint32_t>(sw)) : kNoExp;
      excl = max(excl, block_max_int<6>(val, lane));
      if (prefix & upto) break;
      p -= 64;
    }
    if (lane == 0) {
      __hip_atomic_store(&status[tile], pack_state(kPrefix, max(excl, agg)), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      s_excl = excl;
    }
  }
  __syncthreads();
  const int before = max(s_excl, texcl);  // running exponent before this thread's first value

  // codes, and the entries where the running exponent rises
  int64_t m[kAbPT];
  int prev = before;
  int64_t* table = ab_table(work);
#pragma unroll
  for (int k = 0; k < kAbPT; ++k) {
    const int R = max(before, run[k]);
    if (R > prev && R - kAbEmin >= 0 && R - kAbEmin < kAbEtab) table[R - kAbEmin] = i0 + k;  // (always in range for finite x)
    prev = R;
    m[k] = R == kNoExp ? 0 : static_cast<int64_t>(rint(ldexp(v[k], (w - 1) - R)));
  }
  if (i0 < npad) {
    switch (cbits) {
      case 8: store16<8>(codes, i0, m); break;
      case 12: store16<12>(codes, i0, m); break;
      case 16: store16<16>(codes, i0, m); break;
      case 32: store16<32>(codes, i0, m); break;
      default: store16<64>(codes, i0, m); break;
    }
  }
}

// Keep the (at most) w largest exponents that start a block, in increasing
// order; *nblocks = count, or -1 / -2 for non-finite input / a failed scan.
__global__ void k_abfp_finish(void* work, int w, int64_t* starts, int16_t* exps, int32_t* nblocks) {
  if (threadIdx.x != 0) return;
  const AbWork* hdr = static_cast<const AbWork*>(work);
  const int64_t* table = ab_table(work);
  int c = 0;
  for (int k = kAbEtab - 1; k >= 0 && c < w; --k)
    if (table[k] >= 0) ++c;
  int j = c;
  for (int k = kAbEtab - 1; k >= 0 && j > 0; --k)
    if (table[k] >= 0) {
      --j;
      starts[j] = table[k];
      exps[j] = static_cast<int16_t>(k + kAbEmin);
    }
  *nblocks = (hdr->flags & 1u) ? -1 : (hdr->flags & 2u) ? -2 : c;
}

template <int CB>
__device__ __forceinline__ void decode_thread(const char* codes, int64_t i0, int64_t n, const int64_t* st,
                                              const int16_t* ex, int nb, int w, double* x) {
  int64_t m[kAbPT];
  load16<CB>(codes, i0, m);
  int k = -1;  // last kept block starting at or before i0
  while (k + 1 < nb && st[k + 1] <= i0) ++k;
  double v[kAbPT];
#pragma unroll
  for (int t = 0; t < kAbPT; ++t) {
    while (k + 1 < nb && st[k + 1] <= i0 + t) ++k;
    v[t] = k < 0 ? 0.0 : ldexp(static_cast<double>(m[t]), static_cast<int>(ex[k]) - (w - 1));
  }
  if (i0 + kAbPT <= n) {
    __builtin_memcpy(x + i0, v, sizeof(v));
  } else {
#pragma unroll
    for (int t = 0; t < kAbPT; ++t)
      if (i0 + t < n) x[i0 + t] = v[t];
  }
}

__global__ void __launch_bounds__(kAbNT) k_abfp_decode(const char* __restrict__ codes,
                                                       const int64_t* __restrict__ starts,
                                                       const int16_t* __restrict__ exps,
                                                       const int32_t* __restrict__ nblocks, int64_t n, int w,
                                                       int cbits, double* __restrict__ x) {
  __shared__ int64_t s_st[64];
  __shared__ int16_t s_ex[64];
  const int nb = max(0, min(*nblocks, w));
  if (threadIdx.x < nb) {
    s_st[threadIdx.x] = starts[threadIdx.x];
    s_ex[threadIdx.x] = exps[threadIdx.x];
  }
  __syncthreads();
  const int64_t i0 = static_cast<int64_t>(blockIdx.x) * kAbTile + static_cast<int64_t>(kAbPT) * threadIdx.x;
  if (i0 >= n) return;
  switch (cbits) {
    case 8: decode_thread<8>(codes, i0, n, s_st, s_ex, nb, w, x); break;
    case 12: decode_thread<12>(codes, i0, n, s_st, s_ex, nb, w, x); break;
    case 16: decode_thread<16>(codes, i0, n, s_st, s_ex, nb, w, x); break;
    case 32: decode_thread<32>(codes, i0, n, s_st, s_ex, nb, w, x); break;
    default: decode_thread<64>(codes, i0, n, s_st, s_ex, nb, w, x); break;
  }
}

}  // namespace

template <typename T>
void launch_abfp_encode(const T* x, int64_t n, int w, int cbits, void* codes, int64_t* starts, int16_t* exps,
                        int32_t* nblocks, void* work, hipStream_t st) {
  const int64_t tiles = abfp_tiles(n);
  const int64_t words = kAbEtab + tiles + 2;
  hipLaunchKernelGGL(k_abfp_prep, dim3(static_cast<unsigned>(std::min<int64_t>((words + 255) / 256, 4096))),
                     dim3(256), 0, st, work, tiles);
  const double bytes = static_cast<double>(n) * sizeof(T) + static_cast<double>((n + 63) / 64 * 64) * cbits / 8.0;
  if (tiles > 0) {
    if (g_timing != nullptr) g_timing->begin("k_abfp_encode", bytes, st);
    hipLaunchKernelGGL(k_abfp_encode<T>, dim3(static_cast<unsigned>(tiles)), dim3(kAbNT), 0, st, x, n, w, cbits,
                       static_cast<char*>(codes), work);
    if (g_timing != nullptr) g_timing->end(st);
  }
  hipLaunchKernelGGL(k_abfp_finish, dim3(1), dim3(64), 0, st, work, w, starts, exps, nblocks);
}

void launch_abfp_decode(const void* codes, const int64_t* starts, const int16_t* exps, const int32_t* nblocks,
                        int64_t n, int w, int cbits, double* x, hipStream_t st) {
  const double bytes = static_cast<double>(n) * 8.0 + static_cast<double>((n + 63) / 64 * 64) * cbits / 8.0;
  if (g_timing != nullptr) g_timing->begin("k_abfp_decode", bytes, st);
  hipLaunchKernelGGL(k_abfp_decode, dim3(static_cast<unsigned>(abfp_tiles(n))), dim3(kAbNT), 0, st,
                     static_cast<const char*>(codes), starts, exps, nblocks, n, w, cbits, x);
  if (g_timing != nullptr) g_timing->end(st);
}

// Workspace of the allocation-free encode.  In host code `scratch` is a
// host-side stand-in for the device array, not a device address: the address
// on each device comes from hipGetSymbolAddress, taken once per device (with
// that device current) on its first use and kept.  k_abfp_prep clears what
// must start at zero on every call.
static __device__ __align__(256) unsigned char scratch[kAbNoAllocBytes];

void* abfp_static_workspace() {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> address of `scratch` there
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  const auto it = addr.find(dev);
  if (it != addr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return nullptr;
  addr[dev] = ptr;
  return ptr;
}

template void launch_abfp_encode<float>(const float*, int64_t, int, int, void*, int64_t*, int16_t*, int32_t*, void*,
                                        hipStream_t);
template void launch_abfp_encode<double>(const double*, int64_t, int, int, void*, int64_t*, int16_t*, int32_t*,
                                         void*, hipStream_t);

}  // namespace cmg
