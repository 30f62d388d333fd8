// Open-addressing table of a graph's edges for the closure test: one 8-byte
// slot per key min << 32 | max, linear probing, at most half the slots used.
// Alg. phase3b tests closure by matching a wedge's endpoint pair against the
// edge set by key; this table makes that match a lookup that usually reads
// one 128-byte line.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wedge {

constexpr uint64_t kHashEmpty = ~0ULL;  // no edge key has every bit set

// Slot of key x in a table of 2^bits slots: the high bits of a Fibonacci
// multiplication (Knuth, TAOCP vol. 3, 6.4).
__host__ __device__ __forceinline__ uint64_t hash_slot(uint64_t x, int bits) {
  return (x * 0x9E3779B97F4A7C15ULL) >> (64 - bits);
}

__host__ __device__ __forceinline__ uint64_t edge_key(uint32_t a, uint32_t c) {
  const uint32_t lo = a < c ? a : c, hi = a < c ? c : a;
  return ((uint64_t)lo << 32) | hi;
}

// true iff {a, c} is an edge; *probes += slots read.  A built table has
// empty slots (load <= 1/2), so a probe sequence ends at the key or at an
// empty slot; the bound of one pass over the table only guarantees an end.
__device__ __forceinline__ bool hash_has_edge(const uint64_t* __restrict__ table, int bits,
                                              uint32_t a, uint32_t c, uint64_t* probes) {
  const uint64_t key = edge_key(a, c);
  const uint64_t mask = (1ULL << bits) - 1;
  uint64_t s = hash_slot(key, bits);
  for (uint64_t t = 0; t <= mask; ++t) {
    const uint64_t x = table[s];
    ++*probes;
    if (x == key) return true;
    if (x == kHashEmpty) return false;
    s = (s + 1) & mask;
  }
  return false;
}

}  // namespace wedge
