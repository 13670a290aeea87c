// Plane-addressed section access and block quantisation for the fused 3-D
// level kernels.
//
// On a 3-D level with at least 64^3 nodes one z-plane holds 4^l values: a
// whole number of blocks and of 32-bit code words for every container.  A
// value is then addressed by a wave-uniform plane pointer plus a 32-bit
// in-plane offset, which keeps 64-bit index arithmetic out of the kernels.
//
// Block quantisation uses the following fact: with E(a) the exponent that a
// block whose maximum magnitude is a receives (the frexp exponent of a, plus
// one when a rounds up to 2^(w-1) at w bits), E is non-decreasing in a, so
// the block exponent equals the largest E over the block's values.  Each lane
// computes its own E and the block takes an integer maximum over its lanes
// (DPP row reductions plus readlane), which gives the same exponent and codes
// as rounding the block maximum itself.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace cmg {

struct PSec {
  char* codes;           // code stream (values at bit cbits * i)
  int16_t* exps;         // block exponents
  uint32_t plane_bytes;  // 4^l * cbits / 8
  uint32_t plane_blks;   // 4^l / B
  int32_t cbits;         // 8, 12, 16, 32 or 64
  int32_t w;             // width of the stored codes, sign included
  int32_t wq;            // width of a correction's new codes (SecRef::wq, resolved)
};

struct PlanePtr {
  char* c;
  int16_t* e;
};

// Container width of a section: the kernels' compile-time value CB when
// nonzero (every section the kernel reads value by value then shares it,
// which removes the run-time bit arithmetic of the generic path), else the
// section's own.
template <int CB>
__device__ __forceinline__ int cbits_of(const PSec& s) {
  return CB != 0 ? CB : s.cbits;
}

// Whether a code of a kernel with compile-time container CB (0: run-time)
// and straddle flag HI may need more than 32 bits.
template <int CB, bool HI>
constexpr bool may64() {
  return CB == 0 ? HI : CB == 64;
}

// Whether a kernel's compile-time container CB holds whole, aligned codes
// that one load of the container type returns (sign-extended).
template <int CB>
constexpr bool direct_cb() {
  return CB == 8 || CB == 16 || CB == 32;
}

// Plane p >= 0 of a section.
__device__ __forceinline__ PlanePtr plane_of(const PSec& s, int p) {
  const uint32_t up = static_cast<uint32_t>(p);
  return PlanePtr{s.codes + static_cast<uint64_t>(up) * s.plane_bytes, s.exps + static_cast<uint64_t>(up) * s.plane_blks};
}

// Plane p of a section with the compile-time container CB (plane_of when
// CB = 0): the offsets follow from the level, so the kernel needs neither
// the plane size nor the block count of the section.
template <int CB, int LB>
__device__ __forceinline__ PlanePtr plane_at(const PSec& s, int p, int level) {
  if (CB == 0) return plane_of(s, p);
  const uint64_t v = static_cast<uint64_t>(static_cast<uint32_t>(p)) << (2 * level);  // values before plane p
  return PlanePtr{s.codes + ((v * CB) >> 3), s.exps + (v >> LB)};
}

// Raw words and block exponent of in-plane value xy (see RawCode).  Sections
// carry 16 bytes of padding, so the second word is always readable.  With
// HI = true the second word is always loaded (no branch on the container:
// a load under a branch makes the compiler wait for it, and for every
// memory operation issued before it, where the branches join).  With
// HI = false the caller guarantees an 8-, 16- or 32-bit container, whose
// codes never straddle two words: the second word is not loaded and the
// compiler knows it is zero.
template <int LB, bool HI = true>
__device__ __forceinline__ RawCode raw_at(const PlanePtr& pp, uint32_t xy, int cbits) {
  const uint32_t bit = xy * static_cast<uint32_t>(cbits);
  const uint32_t* wp = reinterpret_cast<const uint32_t*>(pp.c + ((bit >> 5) << 2));
  RawCode r;
  r.lo = wp[0];
  r.hi = HI ? wp[1] : 0u;
  r.e = pp.e[xy >> LB];
  return r;
}

// Codes of the pair of values xy0, xy0 + 1 (xy0 even) of a plane whose
// container has at most 32 bits.  Value xy0 starts at bit 0, 8, 16 or 24 of
// its word, so the two codes lie within that word and the next (one 8-byte
// load; the padding covers the word after the last), and they share one
// block exponent (a block holds at least 32 values).
template <int LB>
__device__ __forceinline__ RawCode pair_at(const PlanePtr& pp, uint32_t xy0, int cbits) {
  const uint32_t bit = xy0 * static_cast<uint32_t>(cbits);
  uint2 v;
  __builtin_memcpy(&v, pp.c + ((bit >> 5) << 2), 8);
  return RawCode{v.x, v.y, pp.e[xy0 >> LB]};
}

// The decoders below need no test for the all-zero block: its codes are 0,
// and its sentinel exponent (-32768) would scale any code to zero anyway.

// Value c (0 or 1) of a pair read by pair_at, as float (w <= 24).
__device__ __forceinline__ float pair_f32(const RawCode& r, uint32_t xy0, int c, int cbits, int w) {
  const uint32_t sh = ((xy0 * static_cast<uint32_t>(cbits)) & 31u) + (c != 0 ? static_cast<uint32_t>(cbits) : 0u);
  const bool up = sh >= 32u;
  const uint32_t x = __builtin_amdgcn_alignbit(up ? 0u : r.hi, up ? r.hi : r.lo, sh & 31u);
  const int m = static_cast<int>(x << (32 - cbits)) >> (32 - cbits);
  return ldexpf(static_cast<float>(m), r.e - (w - 1));
}

// pair_at for a compile-time container: with direct_cb<CB>() the two codes
// as one aligned load (CB = 32: lo and hi; 16: the halves of lo; 8: the two
// low bytes of lo), else pair_at.  Read with pair_code_f32.
template <int CB, int LB>
__device__ __forceinline__ RawCode pair_code_at(const PlanePtr& pp, uint32_t xy0, int cbits) {
  if (!direct_cb<CB>()) return pair_at<LB>(pp, xy0, cbits);
  const char* p = pp.c + xy0 * static_cast<uint32_t>(CB / 8);  // 32-bit offset, see code_at
  RawCode r{0u, 0u, pp.e[xy0 >> LB]};
  if (CB == 32) {
    uint2 v;
    __builtin_memcpy(&v, p, 8);
    r.lo = v.x;
    r.hi = v.y;
  } else if (CB == 16) {
    r.lo = *reinterpret_cast<const uint32_t*>(p);
  } else {
    r.lo = *reinterpret_cast<const uint16_t*>(p);
  }
  return r;
}
// Value c (0 or 1) of a pair read by pair_code_at<CB>, as float (w = wm1 + 1).
template <int CB>
__device__ __forceinline__ float pair_code_f32(const RawCode& r, uint32_t xy0, int c, int cbits, int wm1) {
  if (!direct_cb<CB>()) return pair_f32(r, xy0, c, cbits, wm1 + 1);
  int m;
  if (CB == 32) m = static_cast<int>(c != 0 ? r.hi : r.lo);
  else if (CB == 16) m = c != 0 ? static_cast<int>(r.lo) >> 16 : static_cast<int>(r.lo << 16) >> 16;
  else m = c != 0 ? static_cast<int>(r.lo << 16) >> 24 : static_cast<int>(r.lo << 24) >> 24;
  return ldexpf(static_cast<float>(m), r.e - wm1);
}

// Value of a raw code of width w <= 24 (container at most 32 bits) as float:
// the code converts exactly and the scaling rounds once, as the conversion
// of the exact double value to float does.
__device__ __forceinline__ float raw_f32(const RawCode& r, uint32_t xy, int cbits, int w) {
  const uint32_t sh = (xy * static_cast<uint32_t>(cbits)) & 31u;
  const uint32_t x = __builtin_amdgcn_alignbit(r.hi, r.lo, sh);
  const int m = static_cast<int>(x << (32 - cbits)) >> (32 - cbits);
  return ldexpf(static_cast<float>(m), r.e - (w - 1));
}
// The same with wm1 = w - 1 given (a wave-uniform value the caller keeps
// opaque, so that the scaling exponent is one subtraction).
__device__ __forceinline__ float raw_f32_m1(const RawCode& r, uint32_t xy, int cbits, int wm1) {
  const uint32_t sh = (xy * static_cast<uint32_t>(cbits)) & 31u;
  const uint32_t x = __builtin_amdgcn_alignbit(r.hi, r.lo, sh);
  const int m = static_cast<int>(x << (32 - cbits)) >> (32 - cbits);
  return ldexpf(static_cast<float>(m), r.e - wm1);
}

// raw_at for a compile-time container: with direct_cb<CB>() the code itself
// (one 8-, 16- or 32-bit load, sign-extended into lo), else raw_at.  Read
// the result with code_f32.
template <int CB, int LB, bool HI>
__device__ __forceinline__ RawCode code_at(const PlanePtr& pp, uint32_t xy, int cbits) {
  if (!direct_cb<CB>()) return raw_at<LB, HI>(pp, xy, cbits);
  // in-plane byte offsets stay below 2^32 (a plane holds at most 2^24 values
  // here), which keeps the address a 32-bit offset from the plane pointer
  const char* p = pp.c + xy * static_cast<uint32_t>(CB / 8);
  int c;
  if (CB == 8) c = *reinterpret_cast<const int8_t*>(p);
  else if (CB == 16) c = *reinterpret_cast<const int16_t*>(p);
  else c = *reinterpret_cast<const int32_t*>(p);
  return RawCode{static_cast<uint32_t>(c), 0u, pp.e[xy >> LB]};
}
// Value of a code read by code_at<CB> (width w = wm1 + 1 <= 24), as float.
template <int CB>
__device__ __forceinline__ float code_f32(const RawCode& r, uint32_t xy, int cbits, int wm1) {
  if (!direct_cb<CB>()) return raw_f32_m1(r, xy, cbits, wm1);
  return ldexpf(static_cast<float>(static_cast<int>(r.lo)), r.e - wm1);
}

// Exact value of a raw code as double (branch-free: both the 64-bit and the
// narrow reading are formed and one is selected).  With C64 = false the
// caller guarantees a container of at most 32 bits.
template <bool C64 = true>
__device__ __forceinline__ double raw_f64(const RawCode& r, uint32_t xy, int cbits, int w) {
  const uint32_t sh = (xy * static_cast<uint32_t>(cbits)) & 31u;
  const uint32_t x = __builtin_amdgcn_alignbit(r.hi, r.lo, sh);
  double d;
  if (C64) {
    const double d64 = static_cast<double>(static_cast<int64_t>((static_cast<uint64_t>(r.hi) << 32) | r.lo));
    const int sb = cbits == 64 ? 0 : 32 - cbits;
    const double d32 = static_cast<double>(static_cast<int>(x << sb) >> sb);
    d = cbits == 64 ? d64 : d32;
  } else {
    d = static_cast<double>(static_cast<int>(x << (32 - cbits)) >> (32 - cbits));
  }
  return ldexp(d, r.e - (w - 1));
}

// Exact value of a code read by code_at<CB> as double (raw_f64<C64> when
// the container is not direct).
template <int CB, bool C64>
__device__ __forceinline__ double code_f64(const RawCode& r, uint32_t xy, int cbits, int w) {
  if (!direct_cb<CB>()) return raw_f64<C64>(r, xy, cbits, w);
  return ldexp(static_cast<double>(static_cast<int>(r.lo)), r.e - (w - 1));
}

// a * b + c with one rounding, for products that are exact: b is a power of
// two (or zero) and a * b stays in the normal range.  Then the result is the
// separately rounded product and sum, bit for bit, in one instruction.
__device__ __forceinline__ float exact_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double exact_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Hide a per-lane value from loop-invariant code motion, so that values
// derived from it are recomputed where they are used instead of occupying
// registers for the whole z-march.
template <typename T>
__device__ __forceinline__ void opaque(T& v) {
  asm volatile("" : "+v"(v));
}
// The same for a wave-uniform value (kept in scalar registers).
template <typename T>
__device__ __forceinline__ void opaque_s(T& v) {
  asm volatile("" : "+s"(v));
}
// The scalar fields of a section that a kernel with compile-time container
// CB reads (with CB != 0 only the width).
template <int CB = 0>
__device__ __forceinline__ void opaque_sec(PSec& s) {
  if (CB == 0) {
    opaque_s(s.plane_bytes);
    opaque_s(s.plane_blks);
    opaque_s(s.cbits);
  }
  opaque_s(s.w);
}

// ------------------------------------------------------- block exponents
// (dpp_int, block_max_int, exp_lim, lane_exp and kNoExp: device.h)

// Quantise the value of each lane into its block (w <= 24): returns the code,
// *e_out the block exponent (kZeroExp for an all-zero block).
template <int LB>
__device__ __forceinline__ int quant_f32(float v, int w, int lane, int* e_out) {
  const int E = block_max_int<LB>(lane_exp(v, exp_lim(v, w)), lane);
  const int Eq = E == kNoExp ? 0 : E;
  *e_out = E == kNoExp ? kZeroExp : E;
  return static_cast<int>(rintf(ldexpf(v, w - 1 - Eq)));
}

// With W64 = false the caller guarantees w <= 32 (a 32-bit conversion).
template <int LB, bool W64 = true>
__device__ __forceinline__ int64_t quant_f64(double v, int w, int lane, int* e_out) {
  const int E = block_max_int<LB>(lane_exp(v, exp_lim(v, w)), lane);
  const int Eq = E == kNoExp ? 0 : E;
  *e_out = E == kNoExp ? kZeroExp : E;
  const double q = rint(ldexp(v, w - 1 - Eq));
  if (!W64) return static_cast<int64_t>(static_cast<int>(q));
  return w <= 32 ? static_cast<int64_t>(static_cast<int>(q)) : static_cast<int64_t>(q);
}

// The same for R rows at once: every reduction step is taken for all rows
// before the next, so that the rows' independent DPP operations fill each
// other's wait states instead of no-ops.
template <int LB, int R>
__device__ __forceinline__ void block_max_rows(int (&a)[R], int lane) {
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = max(a[r], dpp_int<0xB1>(a[r]));
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = max(a[r], dpp_int<0x4E>(a[r]));
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = max(a[r], dpp_int<0x141>(a[r]));
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = max(a[r], dpp_int<0x140>(a[r]));
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = max(a[r], __builtin_amdgcn_update_dpp(INT32_MIN, a[r], 0x142, 0xA, 0xF, false));
  if (LB == 6) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      a[r] = max(a[r], __builtin_amdgcn_update_dpp(INT32_MIN, a[r], 0x143, 0xC, 0xF, false));
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = __builtin_amdgcn_readlane(a[r], 63);
    return;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int h0 = __builtin_amdgcn_readlane(a[r], 31), h1 = __builtin_amdgcn_readlane(a[r], 63);
    a[r] = lane < 32 ? h0 : h1;
  }
}

// quant_f32 / quant_f64 of R rows at once (the same codes and exponents).
template <int LB, int R>
__device__ __forceinline__ void quant_f32_rows(const float (&v)[R], int w, int lane, int (&m)[R], int (&e)[R]) {
  int E[R];
#pragma unroll
  for (int r = 0; r < R; ++r) E[r] = lane_exp(v[r], exp_lim(v[r], w));
  block_max_rows<LB, R>(E, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int Eq = E[r] == kNoExp ? 0 : E[r];
    e[r] = E[r] == kNoExp ? kZeroExp : E[r];
    m[r] = static_cast<int>(rintf(ldexpf(v[r], w - 1 - Eq)));
  }
}
template <int LB, bool W64, int R>
__device__ __forceinline__ void quant_f64_rows(const double (&v)[R], int w, int lane, int64_t (&m)[R], int (&e)[R]) {
  int E[R];
#pragma unroll
  for (int r = 0; r < R; ++r) E[r] = lane_exp(v[r], exp_lim(v[r], w));
  block_max_rows<LB, R>(E, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int Eq = E[r] == kNoExp ? 0 : E[r];
    e[r] = E[r] == kNoExp ? kZeroExp : E[r];
    const double q = rint(ldexp(v[r], w - 1 - Eq));
    m[r] = !W64 || w <= 32 ? static_cast<int64_t>(static_cast<int>(q)) : static_cast<int64_t>(q);
  }
}

// Store the codes of one row of 64 values (in-plane offset xy0, a multiple
// of 64) held by the 64 lanes.  In the 12-bit container two values take
// three bytes: each even lane joins its code with its odd neighbour's (one
// DPP move) and writes the three bytes as a byte and an aligned short.
// Byte offsets are formed in 32 bits (a plane holds at most 2^24 values), so
// that the store addresses the plane pointer plus a 32-bit offset.
__device__ __forceinline__ void store_row(char* pc, uint32_t xy0, int lane, int64_t m, int cbits) {
  const uint32_t i = xy0 + static_cast<uint32_t>(lane);
  switch (cbits) {
    case 8: *reinterpret_cast<int8_t*>(pc + i) = static_cast<int8_t>(m); break;
    case 16: *reinterpret_cast<int16_t*>(pc + 2u * i) = static_cast<int16_t>(m); break;
    case 32: *reinterpret_cast<int32_t*>(pc + 4u * i) = static_cast<int32_t>(m); break;
    case 64: *reinterpret_cast<int64_t*>(pc + 8u * i) = m; break;
    default: {
      const int c = static_cast<int>(m) & 0xFFF;
      const uint32_t p24 = static_cast<uint32_t>(c) | (static_cast<uint32_t>(dpp_int<0xB1>(c)) << 12);
      if ((lane & 1) == 0) {
        const int i = lane >> 1;  // pair i: bytes 3 i .. 3 i + 2 of the row
        char* b = pc + static_cast<size_t>(xy0 >> 6) * 96 + 3 * i;
        const bool odd = (i & 1) != 0;  // 3 i odd: byte, then short at 3 i + 1
        *reinterpret_cast<uint8_t*>(b + (odd ? 0 : 2)) = static_cast<uint8_t>(odd ? p24 : p24 >> 16);
        *reinterpret_cast<uint16_t*>(b + (odd ? 1 : 0)) = static_cast<uint16_t>(odd ? p24 >> 8 : p24);
      }
    }
  }
}

}  // namespace cmg
