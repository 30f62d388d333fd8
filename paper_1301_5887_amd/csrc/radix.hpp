// LSD radix sort of uint64 keys over chosen 8-bit digits (stable per pass),
// used for the adjacency (keys made from the edge list) and for the centre
// order of the sampling index (degree keys).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "scan.hpp"

namespace wedge {

// ------------------------------------------------------------------ onesweep
// LSD radix sort with one read and one write of the keys per digit: every
// digit's global histogram comes from a single counting pass, and each tile
// finds the keys of its digit in earlier tiles by a decoupled look-back
// (each tile publishes its own digit counts, then walks back over earlier
// tiles' published counts until it meets an inclusive prefix).  Tiles are
// handed out by a ticket counter, so every tile a look-back waits on is
// already running and publishes without waiting on anything.
constexpr int kOsWG = 512;
constexpr int kOsItems = 16;
constexpr int kOsTile = kOsWG * kOsItems;  // 8192 keys, 64 KB in LDS
constexpr int kOsMaxPasses = 8;

// Status word of (tile, digit): pass tag (8 bits) | flag (2) | count (54).
constexpr uint64_t kOsAgg = 1ULL << 54;
constexpr uint64_t kOsInc = 2ULL << 54;
constexpr uint64_t kOsValue = (1ULL << 54) - 1;
// Narrow status word, used by a pass whose every digit holds fewer than 2^26
// keys (so every count and prefix fits): pass tag (4 bits) | flag (2) |
// count (26).  It halves the look-back's status traffic.
constexpr uint32_t kOs32Agg = 1u << 26;
constexpr uint32_t kOs32Inc = 2u << 26;
constexpr uint32_t kOs32Value = (1u << 26) - 1;

struct OsScratch {
  uint64_t* hist;                // [kOsMaxPasses][256] global digit counts
  uint64_t* base;                // [kOsMaxPasses][256] exclusive prefix over digits
  unsigned long long* tickets;   // [kOsMaxPasses] per pass, then a count of stalled look-backs
  uint32_t* narrow;              // [kOsMaxPasses] 1: the pass uses the narrow status words
  unsigned long long* status;    // [tiles][256]
  unsigned int* status32;        // [tiles][256], narrow passes
};

inline uint64_t os_tiles(uint64_t N) { return ceil_div(N, kOsTile); }
inline size_t os_scratch_bytes(uint64_t N) {
  uint64_t t = os_tiles(N);
  if (t == 0) t = 1;
  return round_up(kOsMaxPasses * 256 * 8, 256) * 2 + 256 + 256 + round_up(t * 256 * 8, 256) +
         round_up(t * 256 * 4, 256);
}
inline OsScratch os_scratch(void* p, uint64_t N) {
  uint64_t t = os_tiles(N);
  if (t == 0) t = 1;
  char* c = (char*)p;
  OsScratch s;
  s.hist = (uint64_t*)c;
  c += round_up(kOsMaxPasses * 256 * 8, 256);
  s.base = (uint64_t*)c;
  c += round_up(kOsMaxPasses * 256 * 8, 256);
  s.tickets = (unsigned long long*)c;
  c += 256;
  s.narrow = (uint32_t*)c;
  c += 256;
  s.status = (unsigned long long*)c;
  c += round_up(t * 256 * 8, 256);
  s.status32 = (unsigned int*)c;
  return s;
}

// Directed keys of an edge list: key 2i = u<<ks|w and key 2i+1 = w<<ks|u of
// edge i = (u, w); in a batch (G > 1) ids are local to their graph and are
// shifted by its vertex offset; an edge with an id out of range becomes the
// self-loop 0<<ks|0 (dropped later) and is counted once.
struct EdgeSource {
  const uint32_t* src;
  const uint32_t* dst;
  uint64_t m_in;
  uint32_t n;
  const uint64_t* eoff;  // [G + 1] edge offsets (G > 1)
  const uint32_t* voff;  // [G + 1] vertex offsets (G > 1)
  uint32_t G;
  unsigned long long* rejected;
  // bit position of the source id in a key (key = u << ks | w).  24 (every
  // id < 2^24): 48-bit keys, stored packed as a uint32 array of their low
  // words followed by a uint16 array of their high words, so a pass moves 6
  // bytes per key instead of 8; above 24 (ks = the ids' bit width, so the key
  // has no unused bits between the two ids): keys stored as uint64.
  int ks = 32;
};

// Key i of a sorted array in either layout.
struct KeyView {
  const uint64_t* k;  // 64-bit keys, or the packed layout's base
  uint64_t N;
  int ks;
  __device__ __forceinline__ uint64_t operator[](uint64_t i) const {
    if (ks > 24) return k[i];
    const uint32_t* lo = (const uint32_t*)k;
    const uint16_t* hi = (const uint16_t*)(lo + N);
    return (uint64_t)lo[i] | ((uint64_t)hi[i] << 32);
  }
  __device__ __forceinline__ uint32_t src(uint64_t x) const { return (uint32_t)(x >> ks); }
  __device__ __forceinline__ uint32_t dst(uint64_t x) const {
    return (uint32_t)(x & ((1ULL << ks) - 1));
  }
};

// Sorts the 2 m_in keys of the edges by the digits at `shifts` (least
// significant first).  Pass 0 reads the edges and writes a, later passes
// ping-pong between a and b; *result receives the buffer with the output.
int onesweep_sort_edges(const EdgeSource& E, uint64_t* a, uint64_t* b, const int* shifts,
                        int npass, OsScratch sc, hipStream_t st, uint64_t** result);

// Sorts keys a[0..N) by the digits at `shifts` (least significant first),
// stably, ping-ponging with b; *result receives the buffer with the output.
int onesweep_sort_keys(uint64_t* a, uint64_t* b, uint64_t N, const int* shifts, int npass,
                       OsScratch sc, hipStream_t st, uint64_t** result);

// The centre order of one graph straight from its row starts: vertices of
// degree d < kRowsDirect in order of (d, id) at positions base[d].. of vlist
// (their ids) and vrow (their row starts); the others as keys
// degree << 32 | id, in id order, at big[0..) (their count is the pass's
// count of digit kRowsDirect).
constexpr uint32_t kRowsDirect = 255;
struct RowSink {
  const uint64_t* rowptr;  // [n + 1]
  uint32_t* vlist;         // [n]
  uint64_t* vrow;          // [n]
  uint64_t* big;           // [vertices of degree >= kRowsDirect]
};

// One stable pass over the vertices 0..n-1 by min(degree, kRowsDirect) into
// R; sc.hist[0..256) must hold the counts of that digit.  Leaves the digit
// offsets in sc.base[0..256).
int onesweep_rows(RowSink R, uint64_t n, OsScratch sc, hipStream_t st);

// After a sort on stream st: *target = value if any look-back of that sort
// gave up waiting (its output is then not sorted).  Every tile a look-back
// waits on is already running, so this is not expected; the flag makes it
// visible instead of silent.
int os_flag_stalls(OsScratch sc, uint64_t* target, uint64_t value, hipStream_t st);

}  // namespace wedge
