// wedge_edge_hash_build: the edge table of hash.hpp from a sorted adjacency,
// for the closure test by lookup (wedge_sample_close_hashed).
#include "common.hpp"
#include "hash.hpp"
#include "scan.hpp"

namespace wedge {

constexpr uint64_t kHashChunk = 256;  // adjacency entries per thread

// Every edge {v, w} with v < w inserted once: thread t walks entries
// [t * kHashChunk, (t + 1) * kHashChunk) of col, finding the row of its first
// entry by bisection over rowptr and moving to the next row as it passes a
// row end.
__global__ void k_hash_insert(const uint64_t* __restrict__ rowptr,
                              const uint32_t* __restrict__ col, uint32_t n, uint64_t total,
                              unsigned long long* __restrict__ table, int bits,
                              unsigned long long* __restrict__ full) {
  const uint64_t mask = (1ULL << bits) - 1;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * kHashChunk;
  for (uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kHashChunk; b < total;
       b += stride) {
    const uint64_t e = b + kHashChunk < total ? b + kHashChunk : total;
    uint32_t lo = 0, hi = n;  // last v with rowptr[v] <= b
    while (hi - lo > 1) {
      const uint32_t mid = lo + (hi - lo) / 2;
      if (rowptr[mid] <= b) lo = mid; else hi = mid;
    }
    uint32_t v = lo;
    uint64_t vend = rowptr[v + 1];
    for (uint64_t i = b; i < e; ++i) {
      while (i >= vend && v + 1 < n) vend = rowptr[++v + 1];
      const uint32_t w = col[i];
      if (w <= v) continue;
      const unsigned long long key = ((unsigned long long)v << 32) | w;
      uint64_t s = hash_slot(key, bits);
      uint64_t t = 0;
      for (; t <= mask; ++t) {
        const unsigned long long prev = atomicCAS(&table[s], kHashEmpty, key);
        if (prev == kHashEmpty || prev == key) break;
        s = (s + 1) & mask;
      }
      if (t > mask) atomicAdd(full, 1ULL);  // no empty slot: not expected at load <= 1/2
    }
  }
}

}  // namespace wedge

using namespace wedge;

extern "C" uint32_t wedge_edge_hash_bits(uint64_t m) {
  uint32_t b = 4;
  while (b < 63 && (1ULL << b) < 2 * m) ++b;
  return b;
}

extern "C" int wedge_edge_hash_build(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                     uint64_t m, uint64_t* d_table, uint32_t bits,
                                     uint64_t* d_full, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_edge_hash_build: n must be >= 1");
  if (!d_rowptr || !d_table || !d_full || (m > 0 && !d_col))
    return set_error(WEDGE_EINVAL, "wedge_edge_hash_build: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_table, 8) || !aligned(d_full, 8) ||
      !aligned(d_col, 4))
    return set_error(WEDGE_EINVAL, "wedge_edge_hash_build: misaligned pointer");
  if (bits < 4 || bits > 40 || (1ULL << bits) < 2 * m)
    return set_error(WEDGE_ERANGE, "wedge_edge_hash_build: 2^bits must be >= 2m (bits in [4, 40])");
  hipStream_t st = (hipStream_t)stream;
  int rc = fill<uint64_t>(d_table, 1ULL << bits, kHashEmpty, st);
  if (rc) return rc;
  if ((rc = fill<uint64_t>(d_full, 1, 0, st))) return rc;
  const uint64_t total = 2 * m;
  if (total == 0) return WEDGE_OK;
  uint64_t threads = ceil_div(total, kHashChunk);
  uint64_t blocks = ceil_div(threads, 256);
  if (blocks > 65536) blocks = 65536;
  k_hash_insert<<<(unsigned)blocks, 256, 0, st>>>(d_rowptr, d_col, n, total,
                                                   (unsigned long long*)d_table, (int)bits,
                                                   (unsigned long long*)d_full);
  WEDGE_LAUNCH_CHECK("k_hash_insert");
  return WEDGE_OK;
}
