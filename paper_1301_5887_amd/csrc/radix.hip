// Kernels and driver of the LSD radix sort declared in radix.hpp.
#include "radix.hpp"

namespace wedge {

// ------------------------------------------------------------------ onesweep

struct OsShifts {
  int s[kOsMaxPasses];
  int mirror[kOsMaxPasses];  // pass whose histogram equals this one's, or -1
  int npass;
};

__device__ inline uint32_t os_graph_of_edge(const uint64_t* __restrict__ eoff, uint32_t G,
                                            uint64_t i) {
  uint32_t lo = 0, hi = G;  // last g with eoff[g] <= i
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (eoff[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// The two keys of edge i of the edge list (see EdgeSource): *k0 = u<<ks|w,
// *k1 = w<<ks|u; returns true when an id is out of range.
__device__ inline bool edge_keys(const EdgeSource& E, uint64_t i, uint64_t* k0, uint64_t* k1) {
  uint64_t u = E.src[i], w = E.dst[i];
  uint64_t base = 0, lim = E.n;
  if (E.G > 1) {
    const uint32_t gg = os_graph_of_edge(E.eoff, E.G, i);
    base = E.voff[gg];
    lim = E.voff[gg + 1] - base;
  }
  const bool bad = u >= lim || w >= lim;
  if (bad) {
    u = w = 0;
  } else {
    u += base;
    w += base;
  }
  *k0 = (u << E.ks) | w;
  *k1 = (w << E.ks) | u;
  return bad;
}

// Lanes of the wave, among those with `valid`, whose 8-bit digit equals this
// lane's: each ballot on one digit bit keeps the lanes that agree on it.
// t is 0 or all ones (the bit, sign-extended), so a lane keeps
// p & ~(m ^ t): m where its bit is 1, ~m where it is 0 (one three-input
// bitwise op per 32-bit half).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  const uint64_t v = __ballot(valid);
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  uint32_t t[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) t[b] = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
  // opaque to the optimiser, so each ballot compares t[b] itself instead of
  // re-deriving the bit with a shift
  asm("" : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]),
      "+v"(t[7]));
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t m = __ballot(t[b] != 0);
    lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m, t[b], 0x90);
    hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m >> 32), t[b], 0x90);
  }
  return ((uint64_t)hi << 32) | lo;
}

// Counts of every digit of every pass over all keys, and the rejected edges.
__global__ __launch_bounds__(kOsWG) void k_os_hist_edges(EdgeSource E, OsShifts S,
                                                         uint64_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kOsMaxPasses][256];
  const int tid = threadIdx.x;
  for (int i = tid; i < kOsMaxPasses * 256; i += kOsWG) (&s_h[0][0])[i] = 0;
  __syncthreads();
  unsigned long long bad_edges = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kOsWG;
  auto count = [&](uint64_t k0, uint64_t k1) {
    for (int p = 0; p < S.npass; ++p) {
      if (S.mirror[p] >= 0) continue;
      atomicAdd(&s_h[p][(k0 >> S.s[p]) & 255], 1u);
      atomicAdd(&s_h[p][(k1 >> S.s[p]) & 255], 1u);
    }
  };
  uint64_t i0 = 0;  // edges before i0 are counted by the 16-byte loads
  if (E.G == 1 && ((((uintptr_t)E.src) | ((uintptr_t)E.dst)) & 15) == 0) {
    // four edges per lane and load (the same keys edge_keys makes)
    const uint64_t nq = E.m_in / 4;
    for (uint64_t q = (uint64_t)blockIdx.x * kOsWG + tid; q < nq; q += stride) {
      const uint4 su = reinterpret_cast<const uint4*>(E.src)[q];
      const uint4 du = reinterpret_cast<const uint4*>(E.dst)[q];
      const uint32_t us[4] = {su.x, su.y, su.z, su.w}, ws[4] = {du.x, du.y, du.z, du.w};
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        uint64_t u = us[h], w = ws[h];
        if (u >= E.n || w >= E.n) {
          u = w = 0;
          ++bad_edges;
        }
        count((u << E.ks) | w, (w << E.ks) | u);
      }
    }
    i0 = nq * 4;
  }
  for (uint64_t i = i0 + (uint64_t)blockIdx.x * kOsWG + tid; i < E.m_in; i += stride) {
    uint64_t k0, k1;
    bad_edges += edge_keys(E, i, &k0, &k1) ? 1 : 0;
    count(k0, k1);
  }
  bad_edges = wave_sum<unsigned long long>(bad_edges);
  if ((tid & 63) == 0 && bad_edges) atomicAdd(E.rejected, bad_edges);
  __syncthreads();
  for (int i = tid; i < S.npass * 256; i += kOsWG) {
    const uint32_t c = (&s_h[0][0])[i];
    if (c) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)c);
  }
}

// Copies of each LDS digit counter in k_os_hist_keys: lane group lane / 8
// adds to its own copy.  Its keys (degrees with vertex ids) put most of a
// wave's lanes on the same few digit values, so one copy serialises the adds
// on the same words; with eight copies the bins phase of 2^28 vertices went
// from 13.8 to 11.6 ms.  (The edge keys' digits are spread evenly, and copies
// made that histogram slower.)
constexpr int kHistCopies = 8;

// Counts of every digit of every pass over keys[0..N).
__global__ __launch_bounds__(kOsWG) void k_os_hist_keys(const uint64_t* __restrict__ keys,
                                                        uint64_t N, OsShifts S,
                                                        uint64_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kOsMaxPasses][256][kHistCopies];
  const int tid = threadIdx.x;
  const int cp = (tid & 63) >> 3;
  for (int i = tid; i < kOsMaxPasses * 256 * kHistCopies; i += kOsWG) (&s_h[0][0][0])[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * kOsWG;
  for (uint64_t i = (uint64_t)blockIdx.x * kOsWG + tid; i < N; i += stride) {
    const uint64_t k = keys[i];
    for (int p = 0; p < S.npass; ++p) atomicAdd(&s_h[p][(k >> S.s[p]) & 255][cp], 1u);
  }
  __syncthreads();
  for (int i = tid; i < S.npass * 256; i += kOsWG) {
    const uint32_t* h = (&s_h[0][0][0]) + (size_t)i * kHistCopies;
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < kHistCopies; ++j) c += h[j];
    if (c) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)c);
  }
}

__global__ void k_os_flag(const unsigned long long* __restrict__ stalls,
                          uint64_t* __restrict__ target, uint64_t value) {
  if (threadIdx.x == 0 && *stalls != 0) *target = value;
}

// base[p][d] = number of keys whose digit p is below d; narrow[p] = 1 when
// every digit of pass p holds fewer than 2^26 keys.
__global__ __launch_bounds__(256) void k_os_base(const uint64_t* __restrict__ hist,
                                                 uint64_t* __restrict__ base,
                                                 uint32_t* __restrict__ narrow, OsShifts S) {
  __shared__ uint64_t s_w[4];
  __shared__ uint32_t s_big[4];
  const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
  for (int p = 0; p < S.npass; ++p) {
    const int hp = S.mirror[p] >= 0 ? S.mirror[p] : p;
    const uint64_t c = hist[hp * 256 + d];
    const uint64_t incl = wave_incl_scan(c, lane);
    const uint64_t big = __ballot(c > (uint64_t)kOs32Value);
    if (lane == 63) s_w[wave] = incl;
    if (lane == 0) s_big[wave] = big != 0;
    __syncthreads();
    uint64_t before = 0;
    for (int w = 0; w < wave; ++w) before += s_w[w];
    base[p * 256 + d] = before + incl - c;
    if (d == 0) narrow[p] = (s_big[0] | s_big[1] | s_big[2] | s_big[3]) ? 0u : 1u;
    __syncthreads();
  }
}

template <class W>
__device__ inline W os_load(const W* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class W>
__device__ inline void os_store(W* p, W v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Status word layouts: wide (pass tag in bits 56..63) and narrow (pass tag in
// bits 28..31); `tag64` is the wide tag (pass + 1) << 56.
template <class W>
struct OsWord;
template <>
struct OsWord<unsigned long long> {
  static constexpr unsigned long long kAgg = kOsAgg, kInc = kOsInc, kValue = kOsValue;
  __device__ static unsigned long long tag(uint64_t tag64) { return tag64; }
};
template <>
struct OsWord<unsigned int> {
  static constexpr unsigned int kAgg = kOs32Agg, kInc = kOs32Inc, kValue = kOs32Value;
  __device__ static unsigned int tag(uint64_t tag64) { return (unsigned int)(tag64 >> 28); }
};

// Tiles a look-back step inspects (status loads in flight per digit).
constexpr int kOsLookTiles = 4;

// Exclusive prefix of digit d over the tiles before `tile`: walk back
// kOsLookTiles tiles per step (that many status loads in flight), adding
// published counts in order until an inclusive prefix is met.  A tile that has not published yet
// is running (tiles are taken in ticket order) and publishes without waiting,
// so the wait ends; the bound only guarantees that the wave exits (counted in
// *stalls).
template <class W>
__device__ inline uint64_t os_lookback(const W* __restrict__ status, uint64_t tile, int d,
                                       W tag, unsigned long long* stalls) {
  using Wd = OsWord<W>;
  uint64_t excl = 0;
  uint64_t t = tile - 1;
  uint32_t spins = 0;
  bool done = false;
  while (!done) {
    const uint64_t nload = t + 1 < (uint64_t)kOsLookTiles ? t + 1 : (uint64_t)kOsLookTiles;
    W xs[kOsLookTiles];
#pragma unroll
    for (int j = 0; j < kOsLookTiles; ++j)
      xs[j] = (uint64_t)j < nload ? os_load(status + (t - j) * 256 + d) : W(0);
    uint64_t used = 0;
#pragma unroll
    for (int j = 0; j < kOsLookTiles; ++j) {
      if (done || used != (uint64_t)j || (uint64_t)j >= nload) continue;
      const W x = xs[j];
      if ((W)(x & ~(Wd::kValue | Wd::kAgg | Wd::kInc)) != tag || (x & (Wd::kAgg | Wd::kInc)) == 0)
        continue;
      excl += x & Wd::kValue;
      ++used;
      if (x & Wd::kInc) done = true;
    }
    if (done) break;
    t -= used;
    if (used < nload) {
      if (++spins > (1u << 24)) {
        atomicAdd(stalls, 1ULL);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return excl;
}

// One digit pass.  kEdges: the input keys are made from the edge list.
// kRows: the keys are min(degree, 255) << 32 | v of the vertices v < N, made
// from R.rowptr, and the output is the centre order (RowSink).
template <bool kEdges, bool kPacked = false, bool kRows = false>
__global__ __launch_bounds__(kOsWG) void k_os_pass(EdgeSource E, const uint64_t* __restrict__ in,
                                                   uint64_t* __restrict__ out, uint64_t N,
                                                   int shift, uint64_t tag,
                                                   const uint64_t* __restrict__ base,
                                                   unsigned long long* __restrict__ status,
                                                   unsigned int* __restrict__ status32,
                                                   const uint32_t* __restrict__ narrow,
                                                   unsigned long long* __restrict__ ticket,
                                                   unsigned long long* __restrict__ stalls,
                                                   RowSink R) {
  constexpr int kWaves = kOsWG / 64;
  __shared__ uint64_t s_keys[kOsTile];
  __shared__ uint32_t s_cnt[kWaves][256];
  __shared__ uint32_t s_spare[kWaves][64];
  __shared__ uint32_t s_tile_off[256];
  __shared__ uint64_t s_glob[256];
  __shared__ uint32_t s_wsum[kWaves];
  __shared__ uint64_t s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < kWaves * 256; i += kOsWG) (&s_cnt[0][0])[i] = 0;
  if (tid == 0) s_tile = atomicAdd(ticket, 1ULL);
  __syncthreads();
  const uint64_t tile = s_tile;
  const uint64_t tbase = tile * kOsTile;

  // Keys of the tile: item it of lane l in wave w is key
  // tbase + (w * kOsItems + it) * 64 + l.  The first pass may take its keys in
  // any order (the edge list has none), so each lane reads whole edges and
  // holds both keys of an edge.
  uint64_t key[kOsItems];
  uint32_t rank[kOsItems];
  bool ok[kOsItems];
  if (kEdges) {
    const uint64_t ebase = tile * (kOsTile / 2);
    const bool pairs = E.G == 1 && ((((uintptr_t)E.src) | ((uintptr_t)E.dst)) & 7) == 0;
    if (pairs) {
      // two consecutive edges per lane and load (8-byte loads of src and dst)
#pragma unroll
      for (int it = 0; it < kOsItems / 4; ++it) {
        const uint64_t e = ebase + (uint64_t)wave * 64 * (kOsItems / 2) + (uint64_t)it * 128 +
                           2 * (uint64_t)lane;
        uint2 su = {0, 0}, du = {0, 0};
        if (e + 1 < E.m_in) {
          su = *reinterpret_cast<const uint2*>(E.src + e);
          du = *reinterpret_cast<const uint2*>(E.dst + e);
        } else if (e < E.m_in) {
          su.x = E.src[e];
          du.x = E.dst[e];
        }
        const uint32_t us[2] = {su.x, su.y}, ws[2] = {du.x, du.y};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool valid = e + h < E.m_in;
          uint64_t u = us[h], w = ws[h];
          if (u >= E.n || w >= E.n) u = w = 0;  // counted by the histogram pass
          key[4 * it + 2 * h] = valid ? ((u << E.ks) | w) : 0;
          key[4 * it + 2 * h + 1] = valid ? ((w << E.ks) | u) : 0;
          ok[4 * it + 2 * h] = ok[4 * it + 2 * h + 1] = valid;
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < kOsItems / 2; ++it) {
        const uint64_t e =
            ebase + (uint64_t)wave * 64 * (kOsItems / 2) + (uint64_t)it * 64 + lane;
        const bool valid = e < E.m_in;
        uint64_t k0 = 0, k1 = 0;
        if (valid) edge_keys(E, e, &k0, &k1);
        key[2 * it] = k0;
        key[2 * it + 1] = k1;
        ok[2 * it] = ok[2 * it + 1] = valid;
      }
    }
  } else if (kRows) {
#pragma unroll
    for (int it = 0; it < kOsItems; ++it) {
      const uint64_t g = tbase + (uint64_t)wave * 64 * kOsItems + (uint64_t)it * 64 + lane;
      ok[it] = g < N;
      uint64_t d = 0;
      if (ok[it]) d = R.rowptr[g + 1] - R.rowptr[g];
      key[it] = ((d < kRowsDirect ? d : (uint64_t)kRowsDirect) << 32) | g;
    }
  } else {
#pragma unroll
    for (int it = 0; it < kOsItems; ++it) {
      const uint64_t g = tbase + (uint64_t)wave * 64 * kOsItems + (uint64_t)it * 64 + lane;
      ok[it] = g < N;
      if (kPacked) {
        const uint32_t* in_lo = (const uint32_t*)in;
        const uint16_t* in_hi = (const uint16_t*)(in_lo + N);
        key[it] = ok[it] ? ((uint64_t)in_lo[g] | ((uint64_t)in_hi[g] << 32)) : 0;
      } else {
        key[it] = ok[it] ? in[g] : 0;
      }
    }
  }
  // rank[it]: the key's position among its wave's keys of the same digit
  // (the waves' counts are combined into tile offsets below).
  if (kEdges) {
    // The edge list has no order to keep, so the first pass ranks each key
    // by an LDS add of 1 on its wave's digit counter: the lanes of one add
    // get distinct counts in an unspecified order.  The later passes are
    // stable and cover every digit, so the sorted result depends on the key
    // values only.
#pragma unroll
    for (int it = 0; it < kOsItems; ++it) {
      const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
      uint32_t* slot = ok[it] ? &s_cnt[wave][d] : &s_spare[wave][lane];
      rank[it] = atomicAdd(slot, ok[it] ? 1u : 0u);
    }
  } else {
    // Stable: key (it, lane) goes after every key of its digit in earlier
    // items and in lower lanes of its item.  Per item, the lowest lane of
    // each digit's group adds the group's size to the wave's counter of that
    // digit (LDS returns the count before it) and the group reads it from
    // that lane.  A wave's LDS operations complete in issue order, so item it
    // sees the counts of items 0..it-1.  The peer masks of all items come
    // first (straight-line code the scheduler can interleave); rank[it] holds
    // below | leader << 8 | size << 16 until the counters are read.  Every
    // lane issues the add, the others adding 0 to a slot of their own, so the
    // adds need no branch.
#pragma unroll
    for (int it = 0; it < kOsItems; ++it) {
      const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
      const uint64_t peers = digit_peers(d, ok[it]);
      const uint32_t below =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                    __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
      const uint32_t leader = (uint32_t)__builtin_ctzll(peers | (1ULL << 63));
      rank[it] = below | (leader << 8) | ((uint32_t)__popcll(peers) << 16);
    }
#pragma unroll
    for (int it = 0; it < kOsItems; ++it) {
      const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
      const uint32_t below = rank[it] & 255, leader = (rank[it] >> 8) & 255;
      const bool lead = ok[it] && below == 0;
      uint32_t* slot = lead ? &s_cnt[wave][d] : &s_spare[wave][lane];
      const uint32_t before = atomicAdd(slot, lead ? rank[it] >> 16 : 0u);
      rank[it] = (uint32_t)__shfl(before, (int)leader, 64) + below;
    }
  }
  __syncthreads();
  uint32_t cnt = 0;           // keys of digit tid in the tile
  uint32_t wex[kWaves] = {};  // keys of digit tid in the waves before w
  if (tid < 256) {
    const int d = tid;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      wex[w] = run;
      run += s_cnt[w][d];
    }
    cnt = run;
    // publish this tile's count before looking back
    if (*narrow)
      os_store(status32 + tile * 256 + d,
               OsWord<unsigned int>::tag(tag) | (tile == 0 ? kOs32Inc : kOs32Agg) | cnt);
    else
      os_store(status + tile * 256 + d,
               (unsigned long long)(tag | (tile == 0 ? kOsInc : kOsAgg) | (uint64_t)cnt));
  }
  // tile-local exclusive offsets of the digits (waves 0..3 hold digits)
  {
    const uint32_t incl = wave_incl_scan(cnt, lane);
    if (lane == 63) s_wsum[wave] = incl;
    __syncthreads();
    if (tid < 256) {
      uint32_t off = incl - cnt;
      for (int w = 0; w < wave; ++w) off += s_wsum[w];
      s_tile_off[tid] = off;
      // each wave's first slot for digit tid in the tile-sorted order
#pragma unroll
      for (int w = 0; w < kWaves; ++w) s_cnt[w][tid] = off + wex[w];
    }
  }
  if (tid < 256) {
    const int d = tid;
    uint64_t excl = 0;
    if (tile > 0) {
      if (*narrow) {
        const unsigned int tag32 = OsWord<unsigned int>::tag(tag);
        excl = os_lookback<unsigned int>(status32, tile, d, tag32, stalls);
        os_store(status32 + tile * 256 + d, tag32 | kOs32Inc | (unsigned int)(excl + cnt));
      } else {
        excl = os_lookback<unsigned long long>(status, tile, d, (unsigned long long)tag, stalls);
        os_store(status + tile * 256 + d, (unsigned long long)(tag | kOsInc | (excl + cnt)));
      }
    }
    s_glob[d] = base[d] + excl - s_tile_off[d];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kOsItems; ++it) {
    if (ok[it]) {
      const uint32_t d = (uint32_t)(key[it] >> shift) & 255;
      s_keys[s_cnt[wave][d] + rank[it]] = key[it];
    }
  }
  __syncthreads();
  const uint64_t valid_n = (N - tbase) < (uint64_t)kOsTile ? (N - tbase) : (uint64_t)kOsTile;
  for (int j = tid; j < (int)valid_n; j += kOsWG) {
    const uint64_t k = s_keys[j];
    const uint32_t d = (uint32_t)(k >> shift) & 255;
    const uint64_t at = s_glob[d] + (uint64_t)j;
    if (at < N) {
      if (kRows) {
        const uint32_t v = (uint32_t)k;
        if (d < kRowsDirect) {
          R.vlist[at] = v;
          R.vrow[at] = R.rowptr[v];
        } else {
          R.big[at - base[kRowsDirect]] = ((R.rowptr[v + 1] - R.rowptr[v]) << 32) | v;
        }
      } else if (kPacked) {
        uint32_t* out_lo = (uint32_t*)out;
        uint16_t* out_hi = (uint16_t*)(out_lo + N);
        out_lo[at] = (uint32_t)k;
        out_hi[at] = (uint16_t)(k >> 32);
      } else {
        out[at] = k;
      }
    }
  }
}

int onesweep_sort_edges(const EdgeSource& E, uint64_t* a, uint64_t* b, const int* shifts,
                        int npass, OsScratch sc, hipStream_t st, uint64_t** result) {
  const uint64_t N = 2 * E.m_in;
  *result = a;
  if (npass > kOsMaxPasses) return set_error(WEDGE_ERANGE, "onesweep: too many passes");
  // the counters (and the stall count os_flag_stalls reads) start at zero
  // even when there is nothing to sort
  int rc = fill<unsigned long long>(sc.tickets, kOsMaxPasses + 1, 0, st);
  if (rc || N == 0 || npass <= 0) return rc;
  const uint64_t nt = os_tiles(N);
  OsShifts S;
  S.npass = npass;
  for (int p = 0; p < kOsMaxPasses; ++p) S.s[p] = p < npass ? shifts[p] : 0;
  // both keys of every edge are sorted, so the src digit at bit ks + s has
  // the same histogram as the dst digit at bit s: count it once
  for (int p = 0; p < kOsMaxPasses; ++p) {
    S.mirror[p] = -1;
    if (p >= npass || S.s[p] < E.ks) continue;
    for (int q = 0; q < npass; ++q)
      if (S.s[q] == S.s[p] - E.ks) S.mirror[p] = q;
  }
  if ((rc = fill<uint64_t>(sc.hist, kOsMaxPasses * 256, 0, st))) return rc;
  if ((rc = fill<unsigned long long>(sc.status, nt * 256, 0, st))) return rc;
  if ((rc = fill<unsigned int>(sc.status32, nt * 256, 0u, st))) return rc;
  {
    uint64_t blocks = ceil_div(E.m_in, (uint64_t)kOsWG * 16);
    if (blocks > 2048) blocks = 2048;
    if (blocks == 0) blocks = 1;
    k_os_hist_edges<<<(unsigned)blocks, kOsWG, 0, st>>>(E, S, sc.hist);
    WEDGE_LAUNCH_CHECK("k_os_hist_edges");
  }
  k_os_base<<<1, 256, 0, st>>>(sc.hist, sc.base, sc.narrow, S);
  WEDGE_LAUNCH_CHECK("k_os_base");
  uint64_t* src = nullptr;
  uint64_t* dst = a;
  for (int p = 0; p < npass; ++p) {
    const uint64_t tag = (uint64_t)(p + 1) << 56;
    const uint64_t* base = sc.base + p * 256;
    const dim3 grid((unsigned)nt), block(kOsWG);
    unsigned long long* stalls = sc.tickets + kOsMaxPasses;
    if (E.ks > 24) {
      if (p == 0)
        k_os_pass<true><<<grid, block, 0, st>>>(E, nullptr, dst, N, shifts[p], tag, base, sc.status,
                                                 sc.status32, sc.narrow + p, sc.tickets + p, stalls, RowSink{});
      else
        k_os_pass<false><<<grid, block, 0, st>>>(E, src, dst, N, shifts[p], tag, base, sc.status,
                                                  sc.status32, sc.narrow + p, sc.tickets + p, stalls, RowSink{});
    } else {
      if (p == 0)
        k_os_pass<true, true><<<grid, block, 0, st>>>(E, nullptr, dst, N, shifts[p], tag, base,
                                                       sc.status, sc.status32, sc.narrow + p,
                                                       sc.tickets + p, stalls, RowSink{});
      else
        k_os_pass<false, true><<<grid, block, 0, st>>>(E, src, dst, N, shifts[p], tag, base,
                                                        sc.status, sc.status32, sc.narrow + p,
                                                        sc.tickets + p, stalls, RowSink{});
    }
    WEDGE_LAUNCH_CHECK("k_os_pass");
    src = dst;
    dst = (dst == a) ? b : a;
  }
  *result = src;
  return WEDGE_OK;
}
int onesweep_sort_keys(uint64_t* a, uint64_t* b, uint64_t N, const int* shifts, int npass,
                       OsScratch sc, hipStream_t st, uint64_t** result) {
  *result = a;
  if (npass > kOsMaxPasses) return set_error(WEDGE_ERANGE, "onesweep: too many passes");
  int rc = fill<unsigned long long>(sc.tickets, kOsMaxPasses + 1, 0, st);
  if (rc || N == 0 || npass <= 0) return rc;
  const uint64_t nt = os_tiles(N);
  OsShifts S;
  S.npass = npass;
  for (int p = 0; p < kOsMaxPasses; ++p) {
    S.s[p] = p < npass ? shifts[p] : 0;
    S.mirror[p] = -1;
  }
  if ((rc = fill<uint64_t>(sc.hist, kOsMaxPasses * 256, 0, st))) return rc;
  if ((rc = fill<unsigned long long>(sc.status, nt * 256, 0, st))) return rc;
  if ((rc = fill<unsigned int>(sc.status32, nt * 256, 0u, st))) return rc;
  {
    uint64_t blocks = ceil_div(N, (uint64_t)kOsWG * 16);
    if (blocks > 2048) blocks = 2048;
    k_os_hist_keys<<<(unsigned)blocks, kOsWG, 0, st>>>(a, N, S, sc.hist);
    WEDGE_LAUNCH_CHECK("k_os_hist_keys");
  }
  k_os_base<<<1, 256, 0, st>>>(sc.hist, sc.base, sc.narrow, S);
  WEDGE_LAUNCH_CHECK("k_os_base");
  const EdgeSource none{nullptr, nullptr, 0, 0, nullptr, nullptr, 1, nullptr};
  uint64_t* src = a;
  uint64_t* dst = b;
  for (int p = 0; p < npass; ++p) {
    const uint64_t tag = (uint64_t)(p + 1) << 56;
    k_os_pass<false><<<(unsigned)nt, kOsWG, 0, st>>>(none, src, dst, N, shifts[p], tag,
                                                      sc.base + p * 256, sc.status, sc.status32,
                                                      sc.narrow + p, sc.tickets + p,
                                                      sc.tickets + kOsMaxPasses, RowSink{});
    WEDGE_LAUNCH_CHECK("k_os_pass");
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return WEDGE_OK;
}

int onesweep_rows(RowSink R, uint64_t n, OsScratch sc, hipStream_t st) {
  if (n == 0) return WEDGE_OK;
  const uint64_t nt = os_tiles(n);
  int rc = fill<unsigned long long>(sc.tickets, kOsMaxPasses + 1, 0, st);
  if (rc) return rc;
  if ((rc = fill<unsigned long long>(sc.status, nt * 256, 0, st))) return rc;
  if ((rc = fill<unsigned int>(sc.status32, nt * 256, 0u, st))) return rc;
  OsShifts S;
  S.npass = 1;
  for (int p = 0; p < kOsMaxPasses; ++p) {
    S.s[p] = 32;
    S.mirror[p] = -1;
  }
  k_os_base<<<1, 256, 0, st>>>(sc.hist, sc.base, sc.narrow, S);
  WEDGE_LAUNCH_CHECK("k_os_base");
  const EdgeSource none{nullptr, nullptr, 0, 0, nullptr, nullptr, 1, nullptr};
  k_os_pass<false, false, true><<<(unsigned)nt, kOsWG, 0, st>>>(
      none, nullptr, nullptr, n, 32, 1ULL << 56, sc.base, sc.status, sc.status32, sc.narrow,
      sc.tickets, sc.tickets + kOsMaxPasses, R);
  WEDGE_LAUNCH_CHECK("k_os_pass");
  return WEDGE_OK;
}

int os_flag_stalls(OsScratch sc, uint64_t* target, uint64_t value, hipStream_t st) {
  k_os_flag<<<1, 64, 0, st>>>(sc.tickets + kOsMaxPasses, target, value);
  WEDGE_LAUNCH_CHECK("k_os_flag");
  return WEDGE_OK;
}

}  // namespace wedge
