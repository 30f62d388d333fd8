// wedge_validate_csr: a device check that an adjacency has the form the rest
// of the path assumes.  The paper's input is an undirected graph without
// repeated edges or self-loops (Sec. 4.1); in the sorted-row form that means
// every row strictly ascending, no vertex in its own row, and w in row v
// exactly when v is in row w.  wedge_build_csr produces that form; a caller
// that brings its own adjacency can check it here (and with WEDGE_VALIDATE=1
// in the environment, wedge_sample_close checks before sampling).
#include <stdlib.h>
#include <string.h>

#include "common.hpp"
#include "scan.hpp"

namespace wedge {

// Last v in [0, n) with rowptr[v] <= i (bisection; any rowptr gives an index
// in range).
__device__ inline uint32_t row_of_entry(const uint64_t* __restrict__ rowptr, uint32_t n,
                                        uint64_t i) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if (rowptr[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// counts[0]: entries not above their predecessor in the row; [1]: self-loops;
// [2]: entries (v, w) whose reverse (w, v) is missing; [3]: structural
// faults (rowptr[0] != 0, rowptr decreasing, rowptr[n] != 2m, an id >= n).
__global__ void k_validate(const uint64_t* __restrict__ rowptr, const uint32_t* __restrict__ col,
                           uint32_t n, uint64_t m, unsigned long long* __restrict__ counts) {
  unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = 2 * m;
  for (uint64_t v = gid; v <= n; v += stride) {
    const uint64_t r = rowptr[v];
    if (v == 0 && r != 0) ++c3;
    if (v > 0 && r < rowptr[v - 1]) ++c3;
    if (v == n && r != total) ++c3;
  }
  for (uint64_t i = gid; i < total; i += stride) {
    const uint32_t v = row_of_entry(rowptr, n, i);
    const uint32_t w = col[i];
    if (w >= n) {
      ++c3;
      continue;
    }
    if (w == v) ++c1;
    const uint64_t start = rowptr[v];
    if (i > start && i > 0 && col[i - 1] >= w) ++c0;
    uint64_t lo = rowptr[w], hi = rowptr[w + 1];
    if (lo > total) lo = total;
    if (hi > total) hi = total;
    if (lo > hi) {
      ++c3;
      continue;
    }
    bool found = false;
    while (lo < hi) {
      const uint64_t mid = lo + (hi - lo) / 2;
      const uint32_t x = col[mid];
      if (x == v) {
        found = true;
        break;
      }
      if (x < v) lo = mid + 1; else hi = mid;
    }
    if (!found) ++c2;
  }
  c0 = wave_sum<unsigned long long>(c0);
  c1 = wave_sum<unsigned long long>(c1);
  c2 = wave_sum<unsigned long long>(c2);
  c3 = wave_sum<unsigned long long>(c3);
  if ((threadIdx.x & 63) == 0) {
    if (c0) atomicAdd(&counts[0], c0);
    if (c1) atomicAdd(&counts[1], c1);
    if (c2) atomicAdd(&counts[2], c2);
    if (c3) atomicAdd(&counts[3], c3);
  }
}

int validate_csr(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                 uint64_t* d_counts, hipStream_t st) {
  int rc = fill<uint64_t>(d_counts, 4, 0, st);
  if (rc) return rc;
  uint64_t work = 2 * m > (uint64_t)n + 1 ? 2 * m : (uint64_t)n + 1;
  uint64_t blocks = ceil_div(work, 256);
  if (blocks > 65536) blocks = 65536;
  k_validate<<<(unsigned)blocks, 256, 0, st>>>(d_rowptr, d_col, n, m,
                                                (unsigned long long*)d_counts);
  WEDGE_LAUNCH_CHECK("k_validate");
  return WEDGE_OK;
}

bool validate_requested() {
  const char* e = getenv("WEDGE_VALIDATE");
  return e && e[0] && strcmp(e, "0") != 0;
}

// With WEDGE_VALIDATE set: run the check with d_counts as scratch, wait for
// it, and report WEDGE_EGRAPH with the counts if any is nonzero.
int validate_or_fail(const char* who, const uint64_t* d_rowptr, const uint32_t* d_col,
                     uint32_t n, uint64_t m, uint64_t* d_counts, hipStream_t st) {
  int rc = validate_csr(d_rowptr, d_col, n, m, d_counts, st);
  if (rc) return rc;
  uint64_t h[4];
  WEDGE_HIP_TRY(hipMemcpyAsync(h, d_counts, sizeof(h), hipMemcpyDeviceToHost, st));
  WEDGE_HIP_TRY(hipStreamSynchronize(st));
  if (h[0] || h[1] || h[2] || h[3])
    return set_error(WEDGE_EGRAPH,
                     "%s: WEDGE_VALIDATE: the adjacency is not a sorted simple undirected graph "
                     "(%llu unsorted or repeated entries, %llu self-loops, %llu one-way entries, "
                     "%llu structural faults)",
                     who, (unsigned long long)h[0], (unsigned long long)h[1],
                     (unsigned long long)h[2], (unsigned long long)h[3]);
  return WEDGE_OK;
}

}  // namespace wedge

using namespace wedge;

extern "C" int wedge_validate_csr(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                  uint64_t m, uint64_t* d_counts, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_validate_csr: n must be >= 1");
  if (!d_rowptr || !d_counts || (m > 0 && !d_col))
    return set_error(WEDGE_EINVAL, "wedge_validate_csr: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_counts, 8) || !aligned(d_col, 4))
    return set_error(WEDGE_EINVAL, "wedge_validate_csr: misaligned pointer");
  return validate_csr(d_rowptr, d_col, n, m, d_counts, (hipStream_t)stream);
}
