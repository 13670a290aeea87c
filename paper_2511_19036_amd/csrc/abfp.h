// Adaptive-exponent BFP codec (abfp.hip): Sec. 6.1.3, Exponents.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cmg {

constexpr int kAbNT = 256, kAbPT = 16, kAbTile = kAbNT * kAbPT;  // values per workgroup tile
constexpr int kAbEmin = -1100, kAbEtab = 2200;  // exponent table: -1100 .. 1099 (float64 spans -1073 .. 1025)

// Workspace of one encode: tile ticket, error flags, the start of the block
// with each exponent, and one look-back status word per tile.
constexpr int64_t abfp_tiles(int64_t n) { return (n + kAbTile - 1) / kAbTile; }
constexpr int64_t abfp_workspace_bytes(int64_t n) { return 16 + 8 * kAbEtab + 8 * abfp_tiles(n); }

// The allocation-free encode (cmg_abfp_encode_noalloc) takes its workspace
// from one static device array per GPU, sized for inputs of up to
// kAbNoAllocMax values (about 4 MiB).  abfp_static_workspace() returns the
// current device's address of that array (nullptr if HIP cannot give it);
// every call on one device shares it.
constexpr int64_t kAbNoAllocMax = int64_t{1} << 31;
constexpr int64_t kAbNoAllocBytes = abfp_workspace_bytes(kAbNoAllocMax);
void* abfp_static_workspace();

// Codes of the first ceil(n/64)*64 values, block list (kept blocks, at most
// `w`), *nblocks (-1: non-finite input, -2: look-back gave up).  Async.
template <typename T>
void launch_abfp_encode(const T* x, int64_t n, int w, int cbits, void* codes, int64_t* starts, int16_t* exps,
                        int32_t* nblocks, void* work, hipStream_t st);
void launch_abfp_decode(const void* codes, const int64_t* starts, const int16_t* exps, const int32_t* nblocks,
                        int64_t n, int w, int cbits, double* x, hipStream_t st);

}  // namespace cmg
