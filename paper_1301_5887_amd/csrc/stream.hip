// wedge_sample_stream: the plain path with the edge list in host memory and
// no adjacency on the device (the paper's setting: the graph is an edge list
// that no single memory holds, and every phase is a pass over it).  The edge
// list streams from host memory in chunks, copies overlapping the kernels:
//  1. degree pass (Alg. phase1a's count; with no repeated edges, Sec. 4.1's
//     input, a count is a degree); the wedges per vertex, the bins and the
//     sampling index follow from the degrees alone (Alg. phase1b);
//  2. every sample's centre and neighbour ranks (i, j) are drawn without an
//     adjacency (the same Philox stream, centre order and pair numbering as
//     wedge_sample_close), the drawn centres are marked, and gather passes
//     collect the edges of marked centres, a vertex range at a time, and sort
//     them into rows, which resolves (i, j) to the endpoints (the Sampling
//     procedure of Alg. phase2c: a centre's reducer sees all its edges);
//  3. one more pass is the closure join (Alg. phase3b, wedge_closure_join);
// then the classes of Alg. phase4c come from the endpoints' streamed degrees.
// For a simple edge list the counts and records equal wedge_sample_close's on
// the adjacency built from the same list.
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "edge_stream.hpp"
#include "radix.hpp"
#include "sample.hpp"
#include "scan.hpp"

namespace wedge {

__global__ void k_stream_degree(const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst,
                                uint64_t ne, uint32_t n, unsigned int* __restrict__ deg,
                                unsigned long long* __restrict__ rejected) {
  unsigned long long bad = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += stride) {
    const uint32_t u = src[i], w = dst[i];
    if (u >= n || w >= n) {
      ++bad;
      continue;
    }
    if (u == w) continue;
    atomicAdd(&deg[u], 1u);
    atomicAdd(&deg[w], 1u);
  }
  bad = wave_sum<unsigned long long>(bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(rejected, bad);
}

// rowptr of the (virtual) adjacency: exclusive prefix of the degrees over
// n + 1 entries, so rowptr[n] = 2m.
struct DegLoad {
  const unsigned int* deg;
  uint32_t n;
  __device__ uint64_t operator()(uint64_t i) const { return i < n ? (uint64_t)deg[i] : 0; }
};
struct RowStore {
  uint64_t* rowptr;
  __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t) const { rowptr[i] = prefix; }
};
// Degrees of the marked vertices only (the keys a gather pass collects).
struct MarkedLoad {
  const unsigned int* deg;
  const uint8_t* flag;
  uint32_t n;
  __device__ uint64_t operator()(uint64_t i) const {
    return (i < n && flag[i]) ? (uint64_t)deg[i] : 0;
  }
};

// Row r of the draws: bin rows_bin[r], records at rows_bin[r] * stride, k
// samples, and its slots [rows_off[r], rows_off[r] + k) of the endpoint and
// closure arrays.
struct DrawRows {
  const uint64_t* k;
  const uint64_t* off;
  const uint32_t* bin;
  uint32_t nrows;
  uint64_t stride;
};

__global__ void k_mark_centres(const wedge_sample_rec* __restrict__ rec, DrawRows R,
                               uint8_t* __restrict__ flag) {
  for (uint32_t r = blockIdx.y; r < R.nrows; r += gridDim.y) {
    const uint64_t k = R.k[r], base = (uint64_t)R.bin[r] * R.stride;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < k;
         s += (uint64_t)gridDim.x * blockDim.x)
      flag[rec[base + s].v] = 1;
  }
}

__global__ void k_marked_max(const unsigned int* __restrict__ deg, const uint8_t* __restrict__ flag,
                             uint32_t n, unsigned int* __restrict__ out) {
  unsigned int mx = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (flag[v]) mx = max(mx, deg[v]);
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (unsigned int)__shfl_xor((int)mx, o, 64));
  if ((threadIdx.x & 63) == 0 && mx) atomicMax(out, mx);
}

// Largest hi in [lo, n] with pre[hi] - pre[lo] <= cap (pre non-decreasing).
__global__ void k_next_cut(const uint64_t* __restrict__ pre, uint32_t n, uint32_t lo, uint64_t cap,
                           uint64_t* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint64_t base = pre[lo];
  uint64_t a = lo, b = n;  // answer in [a, b]
  while (a < b) {
    const uint64_t mid = (a + b + 1) >> 1;
    if (pre[mid] - base <= cap) a = mid; else b = mid - 1;
  }
  *out = a;
}

// Keys u << 32 | w of every edge end u that is marked and in [lo, hi), both
// orientations of each edge.  A workgroup takes kGatherEdges edges per step
// (kGatherPer per thread, strided for coalesced loads) and reserves the slots
// of all its keys with one atomic add on the cursor, placing each thread's
// keys by a prefix over lanes and waves: adds on the one cursor word are
// serialised, so they are kept to one per kGatherEdges edges.
constexpr int kGatherWG = 256;
constexpr int kGatherPer = 4;
constexpr uint64_t kGatherEdges = (uint64_t)kGatherWG * kGatherPer;

__global__ __launch_bounds__(kGatherWG) void k_stream_gather(
    const uint32_t* __restrict__ src, const uint32_t* __restrict__ dst, uint64_t ne, uint32_t n,
    const uint8_t* __restrict__ flag, uint32_t lo, uint32_t hi, uint64_t* __restrict__ keys,
    unsigned long long* __restrict__ cursor, uint64_t cap) {
  constexpr int kWaves = kGatherWG / 64;
  __shared__ uint32_t s_wave[kWaves];
  __shared__ unsigned long long s_base;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (uint64_t e0 = (uint64_t)blockIdx.x * kGatherEdges; e0 < ne;
       e0 += (uint64_t)gridDim.x * kGatherEdges) {
    uint32_t u[kGatherPer], w[kGatherPer], take = 0, cnt = 0;  // take: bit 2j u, bit 2j+1 w
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j) {
      const uint64_t i = e0 + (uint64_t)j * kGatherWG + tid;
      u[j] = w[j] = 0;
      if (i < ne) {
        u[j] = src[i];
        w[j] = dst[i];
        if (u[j] < n && w[j] < n && u[j] != w[j]) {
          if (u[j] >= lo && u[j] < hi && flag[u[j]]) take |= 1u << (2 * j);
          if (w[j] >= lo && w[j] < hi && flag[w[j]]) take |= 2u << (2 * j);
        }
      }
    }
    cnt = __popc(take);
    const uint32_t incl = wave_incl_scan<uint32_t>(cnt, lane);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (tid == 0) {
      uint32_t total = 0;
#pragma unroll
      for (int x = 0; x < kWaves; ++x) total += s_wave[x];
      s_base = total ? atomicAdd(cursor, (unsigned long long)total) : 0ULL;
    }
    __syncthreads();
    uint64_t at = s_base + incl - cnt;
    for (int x = 0; x < wave; ++x) at += s_wave[x];
#pragma unroll
    for (int j = 0; j < kGatherPer; ++j) {
      if ((take >> (2 * j)) & 1u) {
        if (at < cap) keys[at] = ((uint64_t)u[j] << 32) | w[j];
        ++at;
      }
      if ((take >> (2 * j + 1)) & 1u) {
        if (at < cap) keys[at] = ((uint64_t)w[j] << 32) | u[j];
        ++at;
      }
    }
    __syncthreads();  // s_wave and s_base are rewritten by the next step
  }
}

// start[u] = position of u's first key in the sorted keys; equal neighbours
// (a repeated edge) are counted.
__global__ void k_gather_starts(const uint64_t* __restrict__ keys, uint64_t N,
                                uint64_t* __restrict__ start, unsigned long long* __restrict__ dup) {
  unsigned long long d = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const uint64_t x = keys[i];
    const uint64_t p = i ? keys[i - 1] : ~0ULL;
    if (i == 0 || (uint32_t)(p >> 32) != (uint32_t)(x >> 32)) start[(uint32_t)(x >> 32)] = i;
    d += (i > 0 && p == x);
  }
  d = wave_sum<unsigned long long>(d);
  if ((threadIdx.x & 63) == 0 && d) atomicAdd(dup, d);
}

// The endpoints of every drawn wedge whose centre is in [lo, hi): entries i
// and j of the centre's sorted row.
__global__ void k_resolve_pairs(const wedge_sample_rec* __restrict__ rec, DrawRows R, uint32_t lo,
                                uint32_t hi, const uint64_t* __restrict__ keys,
                                const uint64_t* __restrict__ start, uint32_t* __restrict__ qa,
                                uint32_t* __restrict__ qc) {
  for (uint32_t r = blockIdx.y; r < R.nrows; r += gridDim.y) {
    const uint64_t k = R.k[r], off = R.off[r], base = (uint64_t)R.bin[r] * R.stride;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < k;
         s += (uint64_t)gridDim.x * blockDim.x) {
      const wedge_sample_rec x = rec[base + s];
      if (x.v < lo || x.v >= hi) continue;
      const uint64_t b = start[x.v];
      qa[off + s] = (uint32_t)keys[b + x.a];
      qc[off + s] = (uint32_t)keys[b + x.c];
    }
  }
}

// Classes of Alg. phase4c and the per-row tallies; the records get the
// endpoints and the class.
__global__ void k_stream_classes(wedge_sample_rec* __restrict__ rec, DrawRows R, uint32_t max_bins,
                                 uint32_t tau, uint64_t omega, const uint32_t* __restrict__ qa,
                                 const uint32_t* __restrict__ qc,
                                 const uint8_t* __restrict__ closed,
                                 const unsigned int* __restrict__ deg,
                                 unsigned long long* __restrict__ q) {
  for (uint32_t r = blockIdx.y; r < R.nrows; r += gridDim.y) {
    const uint64_t k = R.k[r], off = R.off[r];
    const uint32_t b = R.bin[r];
    const uint64_t base = (uint64_t)b * R.stride;
    const bool global = b == max_bins;
    const uint64_t lo = global ? 0 : bin_lo_deg(b, tau, omega);
    const uint64_t hi = global ? 0 : bin_lo_deg(b + 1, tau, omega);
    unsigned long long c[4] = {0, 0, 0, 0};
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < k;
         s += (uint64_t)gridDim.x * blockDim.x) {
      const uint32_t a = qa[off + s], cc = qc[off + s];
      uint32_t cls = 0;
      if (closed[off + s]) {
        if (global) {
          cls = 3;
        } else {
          const uint64_t da = deg[a], dc = deg[cc];
          cls = 1u + (lo <= da && da < hi ? 1u : 0u) + (lo <= dc && dc < hi ? 1u : 0u);
        }
      }
      c[0] += cls == 0;
      c[1] += cls == 1;
      c[2] += cls == 2;
      c[3] += cls == 3;
      wedge_sample_rec& x = rec[base + s];
      x.a = a;
      x.c = cc;
      x.cls = cls;
    }
    for (int i = 0; i < 4; ++i) {
      const unsigned long long t = wave_sum<unsigned long long>(c[i]);
      if ((threadIdx.x & 63) == 0 && t) atomicAdd(&q[(uint64_t)b * 4 + i], t);
    }
  }
}

// Counter words of the workspace.
enum : int {
  kCtrRejected = 0,
  kCtrCursor = 1,
  kCtrDup = 2,
  kCtrMaxDeg = 3,  // uint32 in a uint64 slot
  kCtrCut = 4,
  kCtrStall = 5,
  kCtrWords = 8
};

struct StreamLayout {
  unsigned int* deg;
  uint64_t* rowptr;
  uint64_t* pre;
  uint64_t* scan;
  void* index;
  void* bins;
  uint8_t* flag;
  uint64_t* start;
  wedge_sample_rec* rec;
  uint64_t* rows_k;
  uint64_t* rows_off;
  uint32_t* rows_bin;
  uint64_t* qdraw;
  uint32_t* qa;
  uint32_t* qc;
  uint8_t* closed;
  uint64_t* keys_a;
  uint64_t* keys_b;
  void* sort;
  unsigned long long* ctr;
  uint32_t* buf[2][2];
  void* join;
  size_t join_bytes;
};

struct StreamSizes {
  uint32_t n;
  uint64_t m_in;
  uint32_t max_bins;
  uint64_t kmax;   // largest row k (the record stride)
  uint64_t ktot;   // all rows' k
  uint64_t gather_cap;
  uint64_t chunk;
};

static size_t stream_layout(const StreamSizes& z, StreamLayout* L, void* base) {
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;  // sizing calls pass no base
    off += round_up(bytes ? bytes : 1, 256);
    return (void*)p;
  };
  const uint64_t rows = (uint64_t)z.max_bins + 1;
  StreamLayout x;
  x.deg = (unsigned int*)take((size_t)z.n * 4);
  x.rowptr = (uint64_t*)take(((size_t)z.n + 1) * 8);
  x.pre = (uint64_t*)take(((size_t)z.n + 1) * 8);
  x.scan = (uint64_t*)take(scan_ws_elems((uint64_t)z.n + 1) * 8);
  x.index = take(index_bytes(z.n, z.m_in, 1, z.max_bins));
  x.bins = take(bins_workspace_bytes(z.n, 1, z.max_bins));
  x.flag = (uint8_t*)take((size_t)z.n);
  x.start = (uint64_t*)take((size_t)z.n * 8);
  x.rec = (wedge_sample_rec*)take((size_t)(rows * z.kmax) * sizeof(wedge_sample_rec));
  x.rows_k = (uint64_t*)take(rows * 8);
  x.rows_off = (uint64_t*)take(rows * 8);
  x.rows_bin = (uint32_t*)take(rows * 4);
  x.qdraw = (uint64_t*)take(rows * 4 * 8);
  x.qa = (uint32_t*)take(z.ktot * 4);
  x.qc = (uint32_t*)take(z.ktot * 4);
  x.closed = (uint8_t*)take(z.ktot);
  x.keys_a = (uint64_t*)take(z.gather_cap * 8);
  x.keys_b = (uint64_t*)take(z.gather_cap * 8);
  x.sort = take(os_scratch_bytes(z.gather_cap));
  x.ctr = (unsigned long long*)take(kCtrWords * 8);
  for (int b = 0; b < 2; ++b)
    for (int j = 0; j < 2; ++j) x.buf[b][j] = (uint32_t*)take(z.chunk * 4);
  x.join_bytes = wedge_closure_join_workspace(z.ktot, z.chunk);
  x.join = take(x.join_bytes);
  if (L) *L = x;
  return off;
}

static unsigned grid_for(uint64_t items, uint64_t cap) {
  uint64_t b = ceil_div(items ? items : 1, 256);
  return (unsigned)(b < cap ? b : cap);
}

template <class T>
static int read_back(T* h, const T* d, size_t count, hipStream_t st) {
  WEDGE_HIP_TRY(hipMemcpyAsync(h, d, count * sizeof(T), hipMemcpyDeviceToHost, st));
  WEDGE_HIP_TRY(hipStreamSynchronize(st));
  return WEDGE_OK;
}

}  // namespace wedge

using namespace wedge;

static uint64_t stream_chunk(uint64_t chunk_edges) { return chunk_edges ? chunk_edges : kEdgeChunk; }

extern "C" size_t wedge_sample_stream_workspace(uint32_t n, uint64_t m_in, uint32_t max_bins,
                                                const uint64_t* h_k, uint64_t k_global,
                                                uint64_t gather_cap, uint64_t chunk_edges) {
  if (max_bins == 0 || max_bins > 4096 || !h_k) return 0;
  StreamSizes z{n, m_in, max_bins, k_global, k_global, gather_cap, stream_chunk(chunk_edges)};
  for (uint32_t b = 0; b < max_bins; ++b) {
    z.kmax = std::max(z.kmax, h_k[b]);
    z.ktot += h_k[b];
  }
  return stream_layout(z, nullptr, nullptr);
}

extern "C" int wedge_sample_stream(const uint32_t* h_src, const uint32_t* h_dst, uint64_t m_in,
                                   uint32_t n, uint32_t tau, uint64_t omega, uint32_t max_bins,
                                   const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                                   uint64_t gather_cap, uint64_t chunk_edges, uint64_t* d_n_b,
                                   uint64_t* d_p_b, uint64_t* d_q, wedge_sample_rec* d_dump,
                                   uint64_t dump_per_bin, uint64_t* h_info, void* d_workspace,
                                   size_t workspace_bytes, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_sample_stream: n must be >= 1");
  if (tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_sample_stream: need tau >= 1 and integer omega >= 2");
  if (max_bins == 0 || max_bins > 4096)
    return set_error(WEDGE_ERANGE, "wedge_sample_stream: max_bins must be in [1, 4096]");
  if ((m_in > 0 && (!h_src || !h_dst)) || !h_k || !d_n_b || !d_p_b || !d_q || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_sample_stream: null pointer");
  if (!aligned(h_src, 4) || !aligned(h_dst, 4) || !aligned(d_n_b, 8) || !aligned(d_p_b, 8) ||
      !aligned(d_q, 8) || !aligned(d_dump, 16) || !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_sample_stream: misaligned pointer");
  if (gather_cap == 0 || gather_cap >= (1ULL << 40))
    return set_error(WEDGE_ERANGE, "wedge_sample_stream: gather_cap must be in [1, 2^40)");
  uint64_t ktot = k_global;
  for (uint32_t b = 0; b < max_bins; ++b) {
    if (h_k[b] > (1ULL << 40))
      return set_error(WEDGE_ERANGE, "wedge_sample_stream: k[%u] above 2^40", b);
    ktot += h_k[b];
  }
  if (k_global > (1ULL << 40) || ktot >= (1ULL << 40))
    return set_error(WEDGE_ERANGE, "wedge_sample_stream: too many samples");
  const size_t need =
      wedge_sample_stream_workspace(n, m_in, max_bins, h_k, k_global, gather_cap, chunk_edges);
  if (workspace_bytes < need)
    return set_error(WEDGE_EWORKSPACE, "wedge_sample_stream: workspace %zu < %zu bytes",
                     workspace_bytes, need);
  hipStream_t st = (hipStream_t)stream;
  const uint64_t chunk = stream_chunk(chunk_edges);
  StreamSizes z{n, m_in, max_bins, 0, ktot, gather_cap, chunk};
  for (uint32_t b = 0; b < max_bins; ++b) z.kmax = std::max(z.kmax, h_k[b]);
  z.kmax = std::max(z.kmax, k_global);
  StreamLayout L;
  stream_layout(z, &L, d_workspace);
  const uint64_t rows = (uint64_t)max_bins + 1;
  int rc;
  if ((rc = fill<unsigned int>(L.deg, n, 0u, st))) return rc;
  if ((rc = fill<unsigned long long>(L.ctr, kCtrWords, 0ULL, st))) return rc;
  if ((rc = fill<uint64_t>(d_q, rows * 4, 0, st))) return rc;

  // 1. degrees, rowptr, bins and the sampling index
  rc = stream_edges(h_src, h_dst, m_in, chunk, L.buf, st,
                    [&](const uint32_t* src, const uint32_t* dst, uint64_t ne) -> int {
                      k_stream_degree<<<grid_for(ne, 4096), 256, 0, st>>>(
                          src, dst, ne, n, L.deg, L.ctr + kCtrRejected);
                      WEDGE_LAUNCH_CHECK("k_stream_degree");
                      return WEDGE_OK;
                    });
  if (rc) return rc;
  if ((rc = scan_apply<uint64_t>(DegLoad{L.deg, n}, RowStore{L.rowptr}, (uint64_t)n + 1, L.scan, st)))
    return rc;
  uint64_t two_m = 0;
  if ((rc = read_back(&two_m, L.rowptr + n, 1, st))) return rc;
  const uint64_t m = two_m / 2;
  if (m > m_in) return set_error(WEDGE_EHIP, "wedge_sample_stream: degree pass miscounted");
  if ((rc = bins_build(L.rowptr, n, m, nullptr, 1, n, tau, omega, max_bins, d_n_b, d_p_b, L.index,
                       L.bins, st)))
    return rc;
  std::vector<uint64_t> p_b(max_bins);
  if ((rc = read_back(p_b.data(), (const uint64_t*)d_p_b, max_bins, st))) return rc;
  {
    uint64_t overflow = 0;
    const IndexHeader* H = (const IndexHeader*)L.index;
    if ((rc = read_back(&overflow, &H->overflow, 1, st))) return rc;
    if (overflow == ~0ULL)
      return set_error(WEDGE_EHIP, "wedge_sample_stream: the centre-order sort gave up waiting");
  }

  // 2. draws: rows with samples, their record and slot offsets
  std::vector<uint64_t> hk(max_bins), rk, roff;
  std::vector<uint32_t> rbin;
  uint64_t p_all = 0, slots = 0;
  for (uint32_t b = 0; b < max_bins; ++b) {
    hk[b] = p_b[b] ? h_k[b] : 0;
    p_all += p_b[b];
  }
  const uint64_t kg = p_all ? k_global : 0;
  for (uint32_t b = 0; b <= max_bins; ++b) {
    const uint64_t k = b == max_bins ? kg : hk[b];
    if (!k) continue;
    rk.push_back(k);
    roff.push_back(slots);
    rbin.push_back(b);
    slots += k;
  }
  const uint32_t nrows = (uint32_t)rk.size();
  uint64_t info[4] = {m, 0, 0, 0};
  if (nrows > 0) {
    WEDGE_HIP_TRY(hipMemcpyAsync(L.rows_k, rk.data(), nrows * 8, hipMemcpyHostToDevice, st));
    WEDGE_HIP_TRY(hipMemcpyAsync(L.rows_off, roff.data(), nrows * 8, hipMemcpyHostToDevice, st));
    WEDGE_HIP_TRY(hipMemcpyAsync(L.rows_bin, rbin.data(), nrows * 4, hipMemcpyHostToDevice, st));
    // the host vectors must outlive the copies, also on an early error return
    WEDGE_HIP_TRY(hipStreamSynchronize(st));
    const DrawRows R{L.rows_k, L.rows_off, L.rows_bin, nrows, z.kmax};
    const uint64_t kmax_used = *std::max_element(rk.begin(), rk.end());
    const dim3 rgrid(grid_for(kmax_used, 2048), nrows);
    if ((rc = sample_draws(L.rowptr, n, m, L.index, max_bins, hk.data(), kg, seed, L.rec, z.kmax,
                           L.qdraw, st)))
      return rc;
    if ((rc = fill<uint8_t>(L.flag, n, 0, st))) return rc;
    k_mark_centres<<<rgrid, 256, 0, st>>>(L.rec, R, L.flag);
    WEDGE_LAUNCH_CHECK("k_mark_centres");
    k_marked_max<<<grid_for(n, 4096), 256, 0, st>>>(L.deg, L.flag, n,
                                                     (unsigned int*)(L.ctr + kCtrMaxDeg));
    WEDGE_LAUNCH_CHECK("k_marked_max");
    if ((rc = scan_apply<uint64_t>(MarkedLoad{L.deg, L.flag, n}, StoreExclusive<uint64_t>{L.pre},
                                   (uint64_t)n + 1, L.scan, st)))
      return rc;
    uint64_t maxdeg = 0, total = 0;
    if ((rc = read_back(&maxdeg, (const uint64_t*)(L.ctr + kCtrMaxDeg), 1, st))) return rc;
    if ((rc = read_back(&total, L.pre + n, 1, st))) return rc;
    maxdeg &= 0xFFFFFFFFULL;
    if (maxdeg > gather_cap)
      return set_error(WEDGE_EWORKSPACE,
                       "wedge_sample_stream: a sampled centre has %llu edges, gather_cap is %llu",
                       (unsigned long long)maxdeg, (unsigned long long)gather_cap);
    // gather rounds over vertex ranges holding at most gather_cap keys each
    const int ib = bit_width((uint64_t)n - 1) ? bit_width((uint64_t)n - 1) : 1;
    int shifts[kOsMaxPasses];
    int np = 0;
    for (int s = 0; s < ib; s += 8) shifts[np++] = s;
    for (int s = 0; s < ib; s += 8) shifts[np++] = 32 + s;
    const OsScratch osc = os_scratch(L.sort, gather_cap);
    uint32_t lo = 0;
    while (lo < n && info[3] < total) {
      k_next_cut<<<1, 64, 0, st>>>(L.pre, n, lo, gather_cap, (uint64_t*)(L.ctr + kCtrCut));
      WEDGE_LAUNCH_CHECK("k_next_cut");
      uint64_t cut = 0;
      if ((rc = read_back(&cut, (const uint64_t*)(L.ctr + kCtrCut), 1, st))) return rc;
      const uint32_t hi = (uint32_t)cut;
      if (hi <= lo) return set_error(WEDGE_EHIP, "wedge_sample_stream: empty gather range");
      uint64_t want[2] = {0, 0};
      if ((rc = read_back(&want[0], L.pre + lo, 1, st))) return rc;
      if ((rc = read_back(&want[1], L.pre + hi, 1, st))) return rc;
      if ((rc = fill<unsigned long long>(L.ctr + kCtrCursor, 1, 0ULL, st))) return rc;
      rc = stream_edges(h_src, h_dst, m_in, chunk, L.buf, st,
                        [&](const uint32_t* src, const uint32_t* dst, uint64_t ne) -> int {
                          uint64_t groups = ceil_div(ne, kGatherEdges);
                          if (groups > 4096) groups = 4096;
                          k_stream_gather<<<(unsigned)groups, kGatherWG, 0, st>>>(
                              src, dst, ne, n, L.flag, lo, hi, L.keys_a, L.ctr + kCtrCursor,
                              gather_cap);
                          WEDGE_LAUNCH_CHECK("k_stream_gather");
                          return WEDGE_OK;
                        });
      if (rc) return rc;
      uint64_t N = 0;
      if ((rc = read_back(&N, (const uint64_t*)(L.ctr + kCtrCursor), 1, st))) return rc;
      if (N != want[1] - want[0])
        return set_error(WEDGE_EHIP,
                         "wedge_sample_stream: gathered %llu keys for [%u, %u), degrees say %llu "
                         "(the edge list changed between passes?)",
                         (unsigned long long)N, lo, hi,
                         (unsigned long long)(want[1] - want[0]));
      uint64_t* sorted = nullptr;
      if ((rc = onesweep_sort_keys(L.keys_a, L.keys_b, N, shifts, np, osc, st, &sorted))) return rc;
      if ((rc = os_flag_stalls(osc, (uint64_t*)(L.ctr + kCtrStall), 1, st))) return rc;
      if (N > 0) {
        k_gather_starts<<<grid_for(N, 8192), 256, 0, st>>>(sorted, N, L.start, L.ctr + kCtrDup);
        WEDGE_LAUNCH_CHECK("k_gather_starts");
        k_resolve_pairs<<<rgrid, 256, 0, st>>>(L.rec, R, lo, hi, sorted, L.start, L.qa, L.qc);
        WEDGE_LAUNCH_CHECK("k_resolve_pairs");
      }
      info[2] += 1;
      info[3] += N;
      lo = hi;
    }

    // 3. closure join against the stream, then classes and tallies
    if ((rc = wedge_closure_join(L.qa, L.qc, slots, h_src, h_dst, m_in, chunk, L.closed, L.join,
                                 L.join_bytes, st)))
      return rc;
    k_stream_classes<<<rgrid, 256, 0, st>>>(L.rec, R, max_bins, tau, omega, L.qa, L.qc, L.closed,
                                            L.deg, (unsigned long long*)d_q);
    WEDGE_LAUNCH_CHECK("k_stream_classes");
    if (d_dump && dump_per_bin > 0) {
      for (uint32_t r = 0; r < nrows; ++r) {
        const uint64_t cnt = std::min(rk[r], dump_per_bin);
        WEDGE_HIP_TRY(hipMemcpyAsync(d_dump + (uint64_t)rbin[r] * dump_per_bin,
                                     L.rec + (uint64_t)rbin[r] * z.kmax,
                                     cnt * sizeof(wedge_sample_rec), hipMemcpyDeviceToDevice, st));
      }
    }
  }
  uint64_t ctr[kCtrWords];
  if ((rc = read_back(ctr, (const uint64_t*)L.ctr, kCtrWords, st))) return rc;
  info[1] = ctr[kCtrRejected];
  if (h_info) memcpy(h_info, info, sizeof(info));
  if (ctr[kCtrStall])
    return set_error(WEDGE_EHIP, "wedge_sample_stream: a row sort gave up waiting");
  if (ctr[kCtrDup])
    return set_error(WEDGE_EGRAPH,
                     "wedge_sample_stream: %llu repeated edges in the sampled centres' rows (the "
                     "edge list must be simple)",
                     (unsigned long long)ctr[kCtrDup]);
  return WEDGE_OK;
}
