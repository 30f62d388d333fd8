// Closure by a join against an unsorted edge stream (the pattern of
// Alg. phase3b): the wedges' endpoint pairs become canonical keys
// min<<32|max in an open-addressing table in HBM; the edge list, held in host
// memory, streams through in chunks (copies on a second stream overlap the
// probes of the previous chunk), and every edge whose key is in the table
// marks it; each wedge then reads its key's mark.  No adjacency is built and
// the edge list is never sorted.
#include <mutex>

#include "common.hpp"
#include "edge_stream.hpp"
#include "scan.hpp"

namespace wedge {

constexpr uint64_t kJoinEmpty = ~0ULL;  // no canonical key of ids < 2^32 - 1
constexpr uint64_t kJoinNone = ~0ULL;

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) as the hash.
__device__ inline uint64_t join_mix(uint64_t x) {
  x ^= x >> 30;
  x *= 0xBF58476D1CE4E5B9ULL;
  x ^= x >> 27;
  x *= 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__device__ inline uint64_t canon_key(uint32_t a, uint32_t c) {
  const uint32_t lo = a < c ? a : c, hi = a < c ? c : a;
  return ((uint64_t)lo << 32) | hi;
}

// Slot of key (inserting it when `insert`), kJoinNone when absent; linear
// probing in a table at most half full, so every probe sequence ends.
template <bool kInsert>
__device__ inline uint64_t join_slot(unsigned long long* table, uint64_t mask, uint64_t key) {
  uint64_t h = join_mix(key) & mask;
  for (;;) {
    const uint64_t cur = __hip_atomic_load(&table[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == key) return h;
    if (cur == kJoinEmpty) {
      if (!kInsert) return kJoinNone;
      const uint64_t prev = atomicCAS(&table[h], (unsigned long long)kJoinEmpty,
                                      (unsigned long long)key);
      if (prev == kJoinEmpty || prev == key) return h;
    }
    h = (h + 1) & mask;
  }
}

__global__ void k_join_insert(const uint32_t* __restrict__ a, const uint32_t* __restrict__ c,
                              uint64_t k, unsigned long long* table, uint64_t mask) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride)
    join_slot<true>(table, mask, canon_key(a[i], c[i]));
}

__global__ void k_join_probe(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             uint64_t ne, unsigned long long* table, uint64_t mask,
                             uint8_t* __restrict__ mark) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
    const uint32_t u = src[i], w = dst[i];
    if (u == w) continue;
    const uint64_t s = join_slot<false>(table, mask, canon_key(u, w));
    if (s != kJoinNone) mark[s] = 1;
  }
}

__global__ void k_join_resolve(const uint32_t* __restrict__ a, const uint32_t* __restrict__ c,
                               uint64_t k, unsigned long long* table, uint64_t mask,
                               const uint8_t* __restrict__ mark, uint8_t* __restrict__ closed) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
    const uint64_t s = join_slot<false>(table, mask, canon_key(a[i], c[i]));
    closed[i] = (s != kJoinNone && mark[s]) ? 1 : 0;
  }
}

static uint64_t join_capacity(uint64_t k) {
  uint64_t cap = 1024;
  while (cap < 2 * k) cap <<= 1;
  return cap;
}

struct JoinWorkspace {
  unsigned long long* table;
  uint8_t* mark;
  uint32_t* buf[2][2];  // [buffer][src, dst]
};

static size_t join_layout(uint64_t k, uint64_t chunk, JoinWorkspace* w, void* base) {
  const uint64_t cap = join_capacity(k);
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;  // sizing calls pass no base
    off += round_up(bytes, 256);
    return p;
  };
  JoinWorkspace x;
  x.table = (unsigned long long*)take(cap * 8);
  x.mark = (uint8_t*)take(cap);
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < 2; ++j) x.buf[b][j] = (uint32_t*)take(chunk * 4);
  if (w) *w = x;
  return off;
}

constexpr uint64_t kJoinChunk = kEdgeChunk;

const char* host_direct(const void* h, size_t bytes) {
  if (!h || bytes == 0) return nullptr;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, h) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a.type != hipMemoryTypeHost || !a.devicePointer) return nullptr;
  void* start = nullptr;
  size_t size = 0;
  if (hipPointerGetAttribute(&start, HIP_POINTER_ATTRIBUTE_RANGE_START_ADDR,
                             (hipDeviceptr_t)h) != hipSuccess ||
      hipPointerGetAttribute(&size, HIP_POINTER_ATTRIBUTE_RANGE_SIZE, (hipDeviceptr_t)h) !=
          hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  const char* p = (const char*)h;
  if (!start || p < (const char*)start || bytes > size ||
      (size_t)(p - (const char*)start) > size - bytes)
    return nullptr;
  return (const char*)a.devicePointer;
}

// Four 16-byte words per thread and step when both addresses are 16-byte
// aligned (many reads in flight over the host link); words otherwise.
constexpr int kCopyWG = 256;
constexpr int kCopyVec = 4;
__global__ __launch_bounds__(kCopyWG) void k_copy_words(const uint32_t* __restrict__ s,
                                                        uint32_t* __restrict__ b, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * kCopyWG;
  const uint64_t t = (uint64_t)blockIdx.x * kCopyWG + threadIdx.x;
  uint64_t i0 = 0;
  if (((((uintptr_t)s) | ((uintptr_t)b)) & 15) == 0) {
    const uint64_t nq = n / 4;
    const uint4* s4 = (const uint4*)s;
    uint4* b4 = (uint4*)b;
    for (uint64_t q = t; q < nq; q += stride * kCopyVec) {
      uint4 x[kCopyVec];
#pragma unroll
      for (int j = 0; j < kCopyVec; ++j) {
        const uint64_t r = q + (uint64_t)j * stride;
        if (r < nq) x[j] = s4[r];
      }
#pragma unroll
      for (int j = 0; j < kCopyVec; ++j) {
        const uint64_t r = q + (uint64_t)j * stride;
        if (r < nq) b4[r] = x[j];
      }
    }
    i0 = nq * 4;
  }
  for (uint64_t i = i0 + t; i < n; i += stride) b[i] = s[i];
}

int copy_words_direct(const uint32_t* s, uint32_t* b, uint64_t n, hipStream_t cs) {
  if (n == 0) return WEDGE_OK;
  uint64_t blocks = ceil_div(n, (uint64_t)kCopyWG * 4 * kCopyVec);
  if (blocks > 2048) blocks = 2048;
  k_copy_words<<<(unsigned)blocks, kCopyWG, 0, cs>>>(s, b, n);
  WEDGE_LAUNCH_CHECK("k_copy_words");
  return WEDGE_OK;
}

int copy_stream(hipStream_t* out, int which) {
  static std::mutex mu;
  static hipStream_t streams[64][2] = {};
  int dev = 0;
  WEDGE_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64 || which < 0 || which > 1)
    return set_error(WEDGE_ERANGE, "copy_stream: device id");
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev][which])
    WEDGE_HIP_TRY(hipStreamCreateWithFlags(&streams[dev][which], hipStreamNonBlocking));
  *out = streams[dev][which];
  return WEDGE_OK;
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_closure_join_workspace(uint64_t k, uint64_t chunk_edges) {
  return join_layout(k, chunk_edges ? chunk_edges : kJoinChunk, nullptr, nullptr);
}

extern "C" int wedge_closure_join(const uint32_t* d_a, const uint32_t* d_c, uint64_t k,
                                  const uint32_t* h_src, const uint32_t* h_dst, uint64_t m_in,
                                  uint64_t chunk_edges, uint8_t* d_closed, void* d_workspace,
                                  size_t workspace_bytes, void* stream) {
  clear_error();
  const uint64_t chunk = chunk_edges ? chunk_edges : kJoinChunk;
  if ((k > 0 && (!d_a || !d_c || !d_closed)) || (m_in > 0 && (!h_src || !h_dst)) || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_closure_join: null pointer");
  if (!aligned(d_a, 4) || !aligned(d_c, 4) || !aligned(h_src, 4) || !aligned(h_dst, 4) ||
      !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_closure_join: misaligned pointer");
  if (k >= (1ULL << 40)) return set_error(WEDGE_ERANGE, "wedge_closure_join: k >= 2^40");
  if (workspace_bytes < wedge_closure_join_workspace(k, chunk_edges))
    return set_error(WEDGE_EWORKSPACE, "wedge_closure_join: workspace %zu < %zu bytes",
                     workspace_bytes, wedge_closure_join_workspace(k, chunk_edges));
  if (k == 0) return WEDGE_OK;
  hipStream_t st = (hipStream_t)stream;
  JoinWorkspace w;
  join_layout(k, chunk, &w, d_workspace);
  const uint64_t cap = join_capacity(k), mask = cap - 1;
  int rc = fill<unsigned long long>(w.table, cap, kJoinEmpty, st);
  if (rc || (rc = fill<uint8_t>(w.mark, cap, 0, st))) return rc;
  k_join_insert<<<2048, 256, 0, st>>>(d_a, d_c, k, w.table, mask);
  WEDGE_LAUNCH_CHECK("k_join_insert");
  rc = stream_edges(h_src, h_dst, m_in, chunk, w.buf, st,
                    [&](const uint32_t* src, const uint32_t* dst, uint64_t ne) -> int {
                      unsigned blocks = (unsigned)((ne + 255) / 256);
                      if (blocks > 4096) blocks = 4096;
                      k_join_probe<<<blocks, 256, 0, st>>>(src, dst, ne, w.table, mask, w.mark);
                      WEDGE_LAUNCH_CHECK("k_join_probe");
                      return WEDGE_OK;
                    });
  if (rc) return rc;
  k_join_resolve<<<2048, 256, 0, st>>>(d_a, d_c, k, w.table, mask, w.mark, d_closed);
  WEDGE_LAUNCH_CHECK("k_join_resolve");
  return WEDGE_OK;
}
