// wedge_build_csr: degree per vertex and sorted adjacency (Alg. phase1a, and
// the input convention of Sec. 4.1 / 5.1: undirected, self-loops and
// repeated edges carry no meaning).
//
// 1. k_canon_keys: each input edge (u, w) becomes the two directed keys
//    u<<32|w and w<<32|u (a self-loop stays a key u<<32|u; an edge with an
//    id >= n becomes the self-loop 0<<32|0 and is counted as rejected).
// 2. LSD radix sort over the significant digits of dst, then of src.
// 3. One fused scan pass: a key is kept iff it is not a self-loop and
//    differs from its predecessor; its exclusive count is its position in
//    col, and every change of src writes the row starts it spans.
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace wedge {

// Graph of edge i of a batch: last g with eoff[g] <= i.
__device__ inline uint32_t graph_of_edge(const uint64_t* __restrict__ eoff, uint32_t G,
                                         uint64_t i) {
  uint32_t lo = 0, hi = G;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (eoff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// Edge i -> the keys u<<32|w and w<<32|u in global ids.  In a batch (G > 1)
// ids are local to their graph and are shifted by the graph's vertex offset.
__global__ void k_canon_keys(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                             uint64_t m_in, uint32_t n, const uint64_t* __restrict__ eoff,
                             const uint32_t* __restrict__ voff, uint32_t G,
                             uint64_t* __restrict__ keys, unsigned long long* __restrict__ rejected) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < m_in; i += stride) {
    uint64_t u = src[i], w = dst[i];
    uint64_t base = 0, lim = n;
    if (G > 1) {
      const uint32_t g = graph_of_edge(eoff, G, i);
      base = voff[g];
      lim = voff[g + 1] - base;
    }
    if (u >= lim || w >= lim) {
      atomicAdd(rejected, 1ULL);
      u = w = 0;
    } else {
      u += base;
      w += base;
    }
    ulonglong2 kv;
    kv.x = (u << 32) | w;
    kv.y = (w << 32) | u;
    reinterpret_cast<ulonglong2*>(keys)[i] = kv;
  }
}

struct DedupLoad {
  const uint64_t* k;
  __device__ uint64_t operator()(uint64_t i) const {
    const uint64_t x = k[i];
    const bool loop = (uint32_t)(x >> 32) == (uint32_t)x;
    const bool repeat = i > 0 && k[i - 1] == x;
    return (!loop && !repeat) ? 1 : 0;
  }
};

struct DedupApply {
  const uint64_t* k;
  uint64_t N;
  uint32_t n;
  uint32_t* col;
  uint64_t* rowptr;
  uint64_t* info;
  __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t keep) const {
    const uint64_t x = k[i];
    const uint32_t s = (uint32_t)(x >> 32);
    if (keep) col[prefix] = (uint32_t)x;
    // rowptr[v] = number of kept keys with src < v: the first key of each
    // src writes it for every vertex since the previous key's src.
    uint64_t first_v;
    if (i == 0) {
      first_v = 0;
    } else {
      const uint32_t sp = (uint32_t)(k[i - 1] >> 32);
      first_v = (sp == s) ? (uint64_t)s + 1 : (uint64_t)sp + 1;
    }
    for (uint64_t v = first_v; v <= s; ++v) rowptr[v] = prefix;
    if (i == N - 1) {
      const uint64_t total = prefix + keep;
      for (uint64_t v = (uint64_t)s + 1; v <= n; ++v) rowptr[v] = total;
      info[0] = total / 2;
    }
  }
};

struct CsrWorkspace {
  uint64_t* keys_a;
  uint64_t* keys_b;
  unsigned long long* counters;
  uint64_t* scan_ws;
  void* radix;
};

static size_t csr_layout(uint64_t m_in, CsrWorkspace* w, void* base) {
  const uint64_t N = 2 * m_in;
  size_t off = 0;
  char* c = (char*)base;
  size_t keys = round_up((N ? N : 1) * 8, 256);
  if (w) w->keys_a = (uint64_t*)(c + off);
  off += keys;
  if (w) w->keys_b = (uint64_t*)(c + off);
  off += keys;
  if (w) w->counters = (unsigned long long*)(c + off);
  off += 256;
  if (w) w->scan_ws = (uint64_t*)(c + off);
  off += round_up(scan_ws_elems(N) * 8, 256);
  if (w) w->radix = (void*)(c + off);
  off += radix_scratch_bytes(N);
  return off;
}

size_t csr_workspace_bytes(uint64_t m_in) { return csr_layout(m_in, nullptr, nullptr); }

int csr_build(const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_in, uint32_t n,
              const uint64_t* d_eoff, const uint32_t* d_voff, uint32_t G, uint64_t* d_rowptr,
              uint32_t* d_col, uint64_t* d_info, void* d_workspace, hipStream_t st) {
  CsrWorkspace w;
  csr_layout(m_in, &w, d_workspace);
  const uint64_t N = 2 * m_in;
  int rc = fill<uint64_t>(d_info, 2, 0, st);
  if (rc) return rc;
  if (N == 0) return fill<uint64_t>(d_rowptr, (uint64_t)n + 1, 0, st);
  {
    uint64_t blocks = ceil_div(m_in, 256);
    if (blocks > 1u << 20) blocks = 1u << 20;
    k_canon_keys<<<(unsigned)blocks, 256, 0, st>>>(d_src, d_dst, m_in, n, d_eoff, d_voff, G,
                                                   w.keys_a, (unsigned long long*)(d_info + 1));
    WEDGE_LAUNCH_CHECK("k_canon_keys");
  }
  // digits of dst (bits 0..nb) then of src (bits 32..32+nb)
  int shifts[16];
  int np = 0;
  const int nb = bit_width((uint64_t)n - 1);
  for (int s = 0; s < nb; s += 8) shifts[np++] = s;
  for (int s = 0; s < nb; s += 8) shifts[np++] = 32 + s;
  uint64_t* sorted = nullptr;
  rc = radix_sort(w.keys_a, w.keys_b, N, shifts, np, radix_scratch(w.radix, N), st, &sorted);
  if (rc) return rc;
  return scan_apply<uint64_t>(DedupLoad{sorted}, DedupApply{sorted, N, n, d_col, d_rowptr, d_info},
                              N, w.scan_ws, st);
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_build_csr_workspace(uint64_t m_in, uint32_t n) {
  (void)n;
  return csr_workspace_bytes(m_in);
}

extern "C" int wedge_build_csr(const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_in,
                               uint32_t n, uint64_t* d_rowptr, uint32_t* d_col, uint64_t* d_info,
                               void* d_workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_build_csr: n must be >= 1");
  if (m_in >= (1ULL << 40)) return set_error(WEDGE_ERANGE, "wedge_build_csr: m_in >= 2^40");
  if (!d_rowptr || !d_info || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_build_csr: null rowptr/info/workspace");
  if (m_in > 0 && (!d_src || !d_dst || !d_col))
    return set_error(WEDGE_EINVAL, "wedge_build_csr: null src/dst/col with m_in > 0");
  if (!aligned(d_rowptr, 8) || !aligned(d_info, 8) || !aligned(d_workspace, 256) ||
      !aligned(d_src, 4) || !aligned(d_dst, 4) || !aligned(d_col, 4))
    return set_error(WEDGE_EINVAL, "wedge_build_csr: misaligned pointer");
  const size_t need = csr_workspace_bytes(m_in);
  if (workspace_bytes < need)
    return set_error(WEDGE_EWORKSPACE, "wedge_build_csr: workspace %zu < %zu bytes",
                     workspace_bytes, need);
  return csr_build(d_src, d_dst, m_in, n, nullptr, nullptr, 1, d_rowptr, d_col, d_info,
                   d_workspace, (hipStream_t)stream);
}
