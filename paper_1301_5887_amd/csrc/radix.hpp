// LSD radix sort of uint64 keys over chosen 8-bit digits (stable per pass).
//
// One pass = per-tile digit histograms (LDS atomics, stored tile-major), a
// column scan of that table (tile offsets for every digit), and a scatter
// kernel that ranks each key stably inside its tile with wave
// ballots (a match mask over the 8 digit bits), reorders the tile in LDS,
// and writes runs of equal digits contiguously so the stores coalesce.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "scan.hpp"

namespace wedge {

constexpr int kRadixWG = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixWG * kRadixItems;  // 4096 keys, 32 KB in LDS

// Scratch for sorting N keys: tile-major histogram (u32) and offset (u64)
// tables [tile][digit], and per-chunk column sums.
struct RadixScratch {
  uint32_t* hist;
  uint64_t* offs;
  uint64_t* scan_ws;
};

inline uint64_t radix_tiles(uint64_t N) { return ceil_div(N, kRadixTile); }
inline size_t radix_scratch_bytes(uint64_t N) {
  uint64_t t = radix_tiles(N);
  if (t == 0) t = 1;
  return round_up(256 * t * 4, 256) + round_up(256 * t * 8, 256) +
         round_up(256 * (ceil_div(t, 256) + 1) * 8, 256);
}
inline RadixScratch radix_scratch(void* p, uint64_t N) {
  uint64_t t = radix_tiles(N);
  if (t == 0) t = 1;
  char* c = (char*)p;
  RadixScratch r;
  r.hist = (uint32_t*)c;
  c += round_up(256 * t * 4, 256);
  r.offs = (uint64_t*)c;
  c += round_up(256 * t * 8, 256);
  r.scan_ws = (uint64_t*)c;
  return r;
}

// Sorts keys[0..N) by the digits at `shifts` (least significant first),
// ping-ponging with alt.  *result receives whichever buffer holds the
// output.
int radix_sort(uint64_t* keys, uint64_t* alt, uint64_t N, const int* shifts, int npass,
               RadixScratch sc, hipStream_t st, uint64_t** result);

}  // namespace wedge
