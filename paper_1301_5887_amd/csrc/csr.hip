// wedge_build_csr: degree per vertex and sorted adjacency (Alg. phase1a, and
// the input convention of Sec. 4.1 / 5.1: undirected, self-loops and
// repeated edges carry no meaning).
//
// 1. Onesweep LSD radix sort of the directed keys u<<ks|w and w<<ks|u of
//    every input edge (u, w) over the significant digits of dst, then of
//    src; ks = 24 when every id is below 2^24 (48-bit keys in the packed
//    layout, 6 bytes moved per key and pass), else 32.  The first pass builds
//    the keys from the edge list as it reads it (a self-loop stays a key
//    u<<ks|u; an edge with an id >= n becomes the self-loop 0 and is counted
//    as rejected).
// 2. One scan over the sorted keys: a key is kept iff it is not a self-loop
//    and differs from its predecessor; its exclusive count is its position
//    in col, and every change of src writes the row starts it spans.
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace wedge {

struct DedupLoad {
  KeyView k;
  __device__ uint64_t operator()(uint64_t i) const {
    const uint64_t x = k[i];
    const bool loop = k.src(x) == k.dst(x);
    const bool repeat = i > 0 && k[i - 1] == x;
    return (!loop && !repeat) ? 1 : 0;
  }
};

// Row starts and compaction over the sorted keys.  Element (it, tid) of a
// tile of kScanTile keys is base + it * 256 + tid (coalesced); every key and
// its predecessor are loaded before the scan, so the writes that follow wait
// on no further loads.
__global__ __launch_bounds__(kScanWG) void k_dedup_apply(const KeyView k, uint64_t N,
                                                         uint32_t n,
                                                         const uint64_t* __restrict__ block_prefix,
                                                         uint32_t* __restrict__ col,
                                                         uint64_t* __restrict__ rowptr,
                                                         uint64_t* __restrict__ info) {
  __shared__ uint64_t s_tot[kScanItems][kScanWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint64_t x[kScanItems], prev[kScanItems];
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kScanWG + tid;
    x[it] = g < N ? k[g] : 0;
    prev[it] = (g > 0 && g < N) ? k[g - 1] : ~0ULL;
  }
  uint32_t keep = 0;  // bit it: key (it, tid) is kept
  uint64_t ex[kScanItems];
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kScanWG + tid;
    const bool loop = k.src(x[it]) == k.dst(x[it]);
    const uint64_t v = (g < N && !loop && x[it] != prev[it]) ? 1 : 0;
    keep |= (uint32_t)v << it;
    const uint64_t incl = wave_incl_scan(v, lane);
    ex[it] = incl - v;
    if (lane == 63) s_tot[it][wave] = incl;
  }
  __syncthreads();
  uint64_t run = block_prefix ? block_prefix[blockIdx.x] : 0;
#pragma unroll
  for (int it = 0; it < kScanItems; ++it) {
    uint64_t row = 0, before = 0;
#pragma unroll
    for (int w = 0; w < kScanWG / 64; ++w) {
      const uint64_t t = s_tot[it][w];
      if (w < wave) before += t;
      row += t;
    }
    const uint64_t g = base + (uint64_t)it * kScanWG + tid;
    if (g < N) {
      const uint64_t prefix = run + before + ex[it];
      const bool kept = (keep >> it) & 1;
      const uint32_t s = k.src(x[it]);
      if (kept) col[prefix] = k.dst(x[it]);
      // rowptr[v] = number of kept keys with src < v: the first key of each
      // src writes it for every vertex since the previous key's src.
      uint64_t first_v;
      if (g == 0) {
        first_v = 0;
      } else {
        const uint32_t sp = k.src(prev[it]);
        first_v = (sp == s) ? (uint64_t)s + 1 : (uint64_t)sp + 1;
      }
      for (uint64_t v = first_v; v <= s; ++v) rowptr[v] = prefix;
      if (g == N - 1) {
        const uint64_t total = prefix + (kept ? 1 : 0);
        for (uint64_t v = (uint64_t)s + 1; v <= n; ++v) rowptr[v] = total;
        info[0] = total / 2;
      }
    }
    run += row;
  }
}

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
  off += os_scratch_bytes(N);
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
  // digits of dst (bits 0..nb) then of src (bits ks..ks+nb); ids below 2^24
  // make 48-bit keys, sorted in the packed layout
  int shifts[16];
  int np = 0;
  const int nb = bit_width((uint64_t)n - 1);
  const int ks = nb <= 24 ? 24 : 32;
  for (int s = 0; s < nb; s += 8) shifts[np++] = s;
  for (int s = 0; s < nb; s += 8) shifts[np++] = ks + s;
  if (np == 0) shifts[np++] = 0;  // n == 1: one pass still writes the keys
  EdgeSource E{d_src, d_dst, m_in, n, d_eoff, d_voff, G, (unsigned long long*)(d_info + 1), ks};
  uint64_t* sorted_base = nullptr;
  const OsScratch osc = os_scratch(w.radix, N);
  rc = onesweep_sort_edges(E, w.keys_a, w.keys_b, shifts, np, osc, st, &sorted_base);
  if (rc) return rc;
  const KeyView sorted{sorted_base, N, ks};
  // kept-key counts per tile, their exclusive scan, then the apply pass
  const uint64_t nb_tiles = ceil_div(N, kScanTile);
  uint64_t* part = w.scan_ws;
  if (nb_tiles == 1) {
    k_dedup_apply<<<1, kScanWG, 0, st>>>(sorted, N, n, nullptr, d_col, d_rowptr, d_info);
    WEDGE_LAUNCH_CHECK("k_dedup_apply");
  } else {
    k_scan_reduce<uint64_t, DedupLoad><<<(unsigned)(nb_tiles + 1), kScanWG, 0, st>>>(
        DedupLoad{sorted}, N, part);
    WEDGE_LAUNCH_CHECK("k_scan_reduce");
    rc = scan_apply<uint64_t>(LoadArray<uint64_t>{part}, StoreExclusive<uint64_t>{part},
                              nb_tiles + 1, part + nb_tiles + 1, st);
    if (rc) return rc;
    k_dedup_apply<<<(unsigned)nb_tiles, kScanWG, 0, st>>>(sorted, N, n, part, d_col, d_rowptr,
                                                          d_info);
    WEDGE_LAUNCH_CHECK("k_dedup_apply");
  }
  // a sort whose bounded wait gave up leaves m = 2^64 - 1
  return os_flag_stalls(osc, d_info, ~0ULL, st);
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
