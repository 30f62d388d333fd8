// wedge_build_csr: degree per vertex and sorted adjacency (Alg. phase1a, and
// the input convention of Sec. 4.1 / 5.1: undirected, self-loops and
// repeated edges carry no meaning).
//
// 1. Onesweep LSD radix sort of the directed keys u<<ks|w and w<<ks|u of
//    every input edge (u, w) over the significant digits of dst, then of
//    src; ks = 24 when every id is below 2^24 (48-bit keys in the packed
//    layout, 6 bytes moved per key and pass), else the ids' bit width (keys
//    of 2 ks bits in uint64, every 8-bit digit of them one pass).  The first pass builds
//    the keys from the edge list as it reads it (a self-loop stays a key
//    u<<ks|u; an edge with an id >= n becomes the self-loop 0 and is counted
//    as rejected).
// 2. One pass over the sorted keys: a key is kept iff it is not a self-loop
//    and differs from its predecessor; its exclusive count is its position
//    in col, and every change of src writes the row starts it spans.
#include <mutex>

#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace wedge {

// Status word of a tile in the dedup's look-back: flag (2 bits) | count.
constexpr uint64_t kDdAgg = 1ULL << 62;
constexpr uint64_t kDdInc = 2ULL << 62;
constexpr uint64_t kDdValue = kDdAgg - 1;

__device__ inline uint64_t dd_load(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void dd_store(unsigned long long* p, uint64_t v) {
  __hip_atomic_store(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Dedup tiles: kDdWG threads with kDdItems keys each.
constexpr int kDdWG = 256;
constexpr int kDdItems = 16;
constexpr uint64_t kDdTile = (uint64_t)kDdWG * kDdItems;

// Row starts and compaction over the sorted keys in one pass.  Tiles of
// kDdTile keys are taken in ticket order; element (it, tid) of a tile is
// base + it * kDdWG + tid (coalesced), and its predecessor is the key of the
// lane below (the wave's lane 0 reads it from memory), so every key is read
// once.  A tile counts its kept keys with ballots, publishes the count and
// finds the kept keys of all earlier tiles by a decoupled look-back (wave 0
// inspects 64 earlier tiles per step), then writes col and the row starts.
__global__ __launch_bounds__(kDdWG) void k_dedup(const KeyView k, uint64_t N, uint32_t n,
                                                   unsigned long long* __restrict__ status,
                                                   unsigned long long* __restrict__ ticket,
                                                   unsigned long long* __restrict__ stalls,
                                                   uint32_t* __restrict__ col,
                                                   uint64_t* __restrict__ rowptr,
                                                   uint64_t* __restrict__ info) {
  constexpr int kWaves = kDdWG / 64;
  __shared__ uint32_t s_tot[kDdItems][kWaves];
  __shared__ uint64_t s_tile, s_excl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_tile = atomicAdd(ticket, 1ULL);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t base = tile * kDdTile;
  uint64_t x[kDdItems], prev[kDdItems];
#pragma unroll
  for (int it = 0; it < kDdItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kDdWG + tid;
    x[it] = g < N ? k[g] : 0;
  }
#pragma unroll
  for (int it = 0; it < kDdItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kDdWG + tid;
    uint64_t p = __shfl_up(x[it], 1, 64);
    if (lane == 0) p = (g > 0 && g < N) ? k[g - 1] : ~0ULL;
    prev[it] = p;
  }
  uint32_t keep = 0;  // bit it: key (it, tid) is kept
  uint32_t ex[kDdItems];  // kept keys of lower lanes in this wave's part of row it
#pragma unroll
  for (int it = 0; it < kDdItems; ++it) {
    const uint64_t g = base + (uint64_t)it * kDdWG + tid;
    const bool loop = k.src(x[it]) == k.dst(x[it]);
    const bool kept = g < N && !loop && x[it] != prev[it];
    const uint64_t m = __ballot(kept);
    ex[it] = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    keep |= (uint32_t)kept << it;
    if (lane == 0) s_tot[it][wave] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (wave == 0) {
    uint64_t part = 0;
    for (int e = lane; e < kDdItems * kWaves; e += 64) part += (&s_tot[0][0])[e];
    const uint64_t agg = wave_sum<uint64_t>(part);
    uint64_t excl = 0;
    if (tile == 0) {
      if (lane == 0) dd_store(status, kDdInc | agg);
    } else {
      if (lane == 0) dd_store(status + tile, kDdAgg | agg);
      // lane l inspects tile t - l; tiles before 0 read as an inclusive 0.
      // Every earlier tile holds its ticket and is running, so each wait
      // ends; the bound only guarantees that the wave exits.
      int64_t t = (int64_t)tile - 1;
      uint32_t spins = 0;
      for (;;) {
        const int64_t j = t - lane;
        const uint64_t sw = j >= 0 ? dd_load(status + j) : kDdInc;
        const uint64_t inc = __ballot((sw & kDdInc) != 0);
        const uint64_t pub = __ballot((sw & (kDdAgg | kDdInc)) != 0);
        const int li = inc ? (int)__builtin_ctzll(inc) : 64;  // nearest inclusive
        const uint64_t upto = li >= 63 ? ~0ULL : ((2ULL << li) - 1);
        if ((pub & upto) != upto) {
          if (++spins > (1u << 24)) {
            if (lane == 0) atomicAdd(stalls, 1ULL);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        excl += wave_sum<uint64_t>(lane <= li ? (sw & kDdValue) : 0);
        if (li < 64) break;
        t -= 64;
      }
      if (lane == 0) dd_store(status + tile, kDdInc | (excl + agg));
    }
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  uint64_t run = s_excl;
#pragma unroll
  for (int it = 0; it < kDdItems; ++it) {
    uint32_t row = 0, before = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = s_tot[it][w];
      if (w < wave) before += c;
      row += c;
    }
    const uint64_t g = base + (uint64_t)it * kDdWG + tid;
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
  if (w) w->scan_ws = (uint64_t*)(c + off);  // the dedup's status word per tile
  off += round_up((ceil_div(N, kDdTile) + 1) * 8, 256);
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
  // Ids below 2^24 make 48-bit keys u << 24 | w, sorted in the packed layout
  // by the digits of dst (bits 0..nb) then of src (bits 24..24+nb).  Wider
  // ids make keys u << nb | w with no unused bits between the ids, sorted by
  // the 8-bit digits of all 2 nb bits (28-bit ids: 7 passes instead of 8).
  int shifts[16];
  int np = 0;
  const int nb = bit_width((uint64_t)n - 1);
  const int ks = nb <= 24 ? 24 : nb;
  if (ks == 24) {
    for (int s = 0; s < nb; s += 8) shifts[np++] = s;
    for (int s = 0; s < nb; s += 8) shifts[np++] = ks + s;
  } else {
    for (int s = 0; s < 2 * nb; s += 8) shifts[np++] = s;
  }
  if (np == 0) shifts[np++] = 0;  // n == 1: one pass still writes the keys
  EdgeSource E{d_src, d_dst, m_in, n, d_eoff, d_voff, G, (unsigned long long*)(d_info + 1), ks};
  uint64_t* sorted_base = nullptr;
  const OsScratch osc = os_scratch(w.radix, N);
  rc = onesweep_sort_edges(E, w.keys_a, w.keys_b, shifts, np, osc, st, &sorted_base);
  if (rc) return rc;
  const KeyView sorted{sorted_base, N, ks};
  // one pass: tiles in ticket order, look-back statuses in the scan scratch
  const uint64_t nb_tiles = ceil_div(N, kDdTile);
  unsigned long long* dd_status = (unsigned long long*)w.scan_ws;
  if ((rc = fill<unsigned long long>(dd_status, nb_tiles, 0, st))) return rc;
  if ((rc = fill<unsigned long long>(w.counters, 1, 0, st))) return rc;
  k_dedup<<<(unsigned)nb_tiles, kDdWG, 0, st>>>(sorted, N, n, dd_status, w.counters,
                                                  osc.tickets + kOsMaxPasses, d_col, d_rowptr,
                                                  d_info);
  WEDGE_LAUNCH_CHECK("k_dedup");
  // a sort or dedup whose bounded wait gave up leaves m = 2^64 - 1
  return os_flag_stalls(osc, d_info, ~0ULL, st);
}

// ------------------------------------------------------ allocation-free form
// The build's workspace, for edge lists of at most kNoAllocMaxEdges input
// edges, as a file-scope device array.  Host code never passes the array's
// name to a kernel (in host code it is a host-side stand-in, not a device
// address): the address comes from hipGetSymbolAddress, taken once per
// device with that device current, and kept per device.  Each device holds
// its own copy of the array until the process ends.
constexpr uint64_t kNoAllocMaxEdges = 1ULL << 20;
constexpr size_t kNoAllocScratchBytes = 36ULL << 20;  // >= csr_workspace_bytes(2^20)
constexpr int kNoAllocMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kNoAllocMaxDevices] = {};

static int scratch_address(void** out) {
  int dev = 0;
  WEDGE_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return set_error(WEDGE_ERANGE, "wedge_build_csr_noalloc: device %d beyond %d", dev,
                     kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    WEDGE_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return set_error(WEDGE_EHIP, "wedge_build_csr_noalloc: no address for the scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return WEDGE_OK;
}

}  // namespace wedge

using namespace wedge;

extern "C" int wedge_build_csr_noalloc(const uint32_t* d_src, const uint32_t* d_dst,
                                       uint64_t m_in, uint32_t n, uint64_t* d_rowptr,
                                       uint32_t* d_col, uint64_t* d_info, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_build_csr_noalloc: n must be >= 1");
  if (m_in > kNoAllocMaxEdges)
    return set_error(WEDGE_EWORKSPACE,
                     "wedge_build_csr_noalloc: m_in = %llu exceeds the %llu input edges its "
                     "static scratch holds",
                     (unsigned long long)m_in, (unsigned long long)kNoAllocMaxEdges);
  if (!d_rowptr || !d_info) return set_error(WEDGE_EINVAL, "wedge_build_csr_noalloc: null rowptr/info");
  if (m_in > 0 && (!d_src || !d_dst || !d_col))
    return set_error(WEDGE_EINVAL, "wedge_build_csr_noalloc: null src/dst/col with m_in > 0");
  if (!aligned(d_rowptr, 8) || !aligned(d_info, 8) || !aligned(d_src, 4) || !aligned(d_dst, 4) ||
      !aligned(d_col, 4))
    return set_error(WEDGE_EINVAL, "wedge_build_csr_noalloc: misaligned pointer");
  if (csr_workspace_bytes(m_in) > kNoAllocScratchBytes)
    return set_error(WEDGE_EWORKSPACE, "wedge_build_csr_noalloc: scratch too small");
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  // every counter and status word the build uses is cleared by the build
  // itself (fill kernels), so the array's previous contents do not matter
  return csr_build(d_src, d_dst, m_in, n, nullptr, nullptr, 1, d_rowptr, d_col, d_info, ws,
                   (hipStream_t)stream);
}

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
