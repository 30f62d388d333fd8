// wedge_bin_counts: wedges per vertex p_v = C(d_v, 2) (Sec. 2.1), vertices
// and wedges per degree bin (Alg. phase1b with Eqs. binlodeg/binid in their
// integer form, Sec. 4.2), and the index the sampler uses to draw a centre
// with probability p_v / p_b (Sec. 3.2).
//
// The index orders vertices by (graph, degree, id) with a stable radix sort
// of the keys g<<gshift | d<<32 | v over the degree and graph digits only.
// Because BinId is monotone in the degree, each bin of each graph is then
// one contiguous run, and within it vertices of equal degree form a "class"
// of equally likely centres: the sampler keeps one cumulative wedge count per
// (graph, distinct degree) instead of one per vertex.  For a single graph
// (G = 1) one stable pass by min(degree, 255) reads the row starts in id
// order and writes the order of every vertex of degree < 255 and its row
// start directly; only the vertices of higher degree (at most 2m / 255) are
// sorted by their degree digits, as keys.
#include <math.h>

#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace wedge {

uint64_t class_capacity(uint64_t n_total, uint64_t m_total, uint32_t G) {
  // In one graph, c distinct positive degrees sum to >= c(c+1)/2 and to
  // <= 2 m_g, so c_g <= sqrt(4 m_g); summed over G graphs (Cauchy-Schwarz)
  // sum_g c_g <= sqrt(4 G M).  Degree 0 and one guard entry add 2 per graph.
  const double s = sqrt(4.0 * (double)G * (double)m_total);
  uint64_t c = (uint64_t)s + 1;
  while (c > 0 && (double)(c - 1) * (double)(c - 1) > 4.0 * (double)G * (double)m_total) --c;
  uint64_t cap = c + 2 * (uint64_t)G + 2;
  if (cap > n_total) cap = n_total;
  return cap ? cap : 1;
}

static size_t index_layout(uint64_t n_total, uint64_t m_total, uint32_t G, uint32_t max_bins,
                           IndexView* v, void* base) {
  const uint64_t cap = class_capacity(n_total, m_total, G);
  char* c = (char*)base;
  size_t off = 0;
  if (v) v->hdr = (IndexHeader*)(c + off);
  off += sizeof(IndexHeader);
  if (v) v->bins = (BinMeta*)(c + off);
  off += round_up(sizeof(BinMeta) * (size_t)G * ((size_t)max_bins + 1), 256);
  if (v) v->vlist = (uint32_t*)(c + off);
  off += round_up((size_t)n_total * 4, 256);
  if (v) v->vrow = (uint64_t*)(c + off);
  off += round_up((size_t)n_total * 8, 256);
  if (v) v->cls_deg = (uint32_t*)(c + off);
  off += round_up(cap * 4, 256);
  if (v) v->cls_start = (uint32_t*)(c + off);
  off += round_up(cap * 4, 256);
  if (v) v->cls_cumw = (uint64_t*)(c + off);
  off += round_up(cap * 8, 256);
  if (v) v->vcode = (uint8_t*)(c + off);
  off += round_up((size_t)n_total, 256);
  if (v) v->vmeta = (uint64_t*)(c + off);
  off += round_up(((size_t)n_total + 1) * 8, 256);
  return off;
}

size_t index_bytes(uint64_t n_total, uint64_t m_total, uint32_t G, uint32_t max_bins) {
  return index_layout(n_total, m_total, G, max_bins, nullptr, nullptr);
}

IndexView index_view(void* base, uint64_t n_total, uint64_t m_total, uint32_t G,
                     uint32_t max_bins) {
  IndexView v;
  index_layout(n_total, m_total, G, max_bins, &v, base);
  return v;
}

// Degree code floor(8 L(d)), L Mitchell's piecewise-linear log2 (0 for
// d = 0): monotone in d, so comparing codes picks the shorter of two rows
// whenever the codes differ.
__device__ inline uint8_t degree_code(uint64_t d) {
  if (d == 0) return 0;
  const uint32_t e = 63 - (uint32_t)__builtin_clzll(d);
  const uint32_t k = 8 * e + (uint32_t)(((d - (1ULL << e)) * 8) >> e);
  return (uint8_t)(k < 255 ? k : 255);
}

__global__ void k_deg_keys(const uint64_t* __restrict__ rowptr, uint32_t n,
                           const uint32_t* __restrict__ voff, uint32_t G, int gshift,
                           uint64_t dmask, uint64_t* __restrict__ keys,
                           uint8_t* __restrict__ vcode, uint64_t* __restrict__ vmeta) {
  uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; v < n; v += stride) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    vcode[v] = degree_code(d);
    vmeta[v] = rowptr[v] | ((uint64_t)degree_code(d) << 56);
    if (v == (uint64_t)n - 1) vmeta[n] = rowptr[n];
    if (d > dmask) d = dmask;
    uint64_t key = (d << 32) | v;
    if (G > 1) key |= (uint64_t)graph_of(voff, G, (uint32_t)v) << gshift;
    keys[v] = key;
  }
}

// *target = value if *word != 0 (after the work before it on the stream).
__global__ void k_flag_if_set(const uint64_t* __restrict__ word, uint64_t* __restrict__ target,
                              uint64_t value) {
  if (threadIdx.x == 0 && *word != 0) *target = value;
}

// One graph: degree code and row word per vertex (as k_deg_keys) and the
// counts of min(degree, kRowsDirect).  Lane group lane / 8 adds to its own
// copy of the counters (most vertices share a few small degrees).
constexpr int kDegCopies = 8;
__global__ __launch_bounds__(256) void k_deg_hist(const uint64_t* __restrict__ rowptr, uint32_t n,
                                                  uint8_t* __restrict__ vcode,
                                                  uint64_t* __restrict__ vmeta,
                                                  uint64_t* __restrict__ hist) {
  __shared__ uint32_t s_h[256][kDegCopies];
  const int tid = threadIdx.x;
  const int cp = (tid & 63) >> 3;
  for (int i = tid; i < 256 * kDegCopies; i += 256) (&s_h[0][0])[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + tid; v < n; v += stride) {
    const uint64_t r0 = rowptr[v], d = rowptr[v + 1] - r0;
    vcode[v] = degree_code(d);
    vmeta[v] = r0 | ((uint64_t)degree_code(d) << 56);
    if (v == (uint64_t)n - 1) vmeta[n] = rowptr[n];
    atomicAdd(&s_h[d < kRowsDirect ? d : kRowsDirect][cp], 1u);
  }
  __syncthreads();
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < kDegCopies; ++j) c += s_h[tid][j];
  if (c) atomicAdd((unsigned long long*)&hist[tid], (unsigned long long)c);
}

// One graph, after the pass by min(degree, kRowsDirect): a class per degree
// d < kRowsDirect that occurs (starting at base[d]), the count and first
// position of the higher-degree vertices, and their key tail big[nbig ..
// bound) set to ~0 so that it sorts last.
__global__ __launch_bounds__(256) void k_rows_classes(const uint64_t* __restrict__ hist,
                                                      const uint64_t* __restrict__ base,
                                                      uint64_t cap, IndexView ix,
                                                      uint64_t* __restrict__ meta) {
  __shared__ uint32_t s_w[4];
  const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
  const bool occ = d < (int)kRowsDirect && hist[d] > 0;
  const uint64_t m = __ballot(occ);
  if (lane == 0) s_w[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t j = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
  for (int w = 0; w < wave; ++w) j += s_w[w];
  if (occ) {
    if (j < cap) {
      ix.cls_deg[j] = (uint32_t)d;
      ix.cls_start[j] = (uint32_t)base[d];
    } else {
      atomicAdd((unsigned long long*)&ix.hdr->overflow, 1ULL);
    }
  }
  if (d == 0) {
    const uint64_t nsmall = (uint64_t)s_w[0] + s_w[1] + s_w[2] + s_w[3];
    meta[0] = hist[kRowsDirect];
    meta[1] = base[kRowsDirect];
    meta[2] = nsmall;
    ix.hdr->num_classes = (uint32_t)(nsmall < cap ? nsmall : cap);
  }
}

__global__ void k_rows_tail(uint64_t* __restrict__ big, uint64_t bound,
                            const uint64_t* __restrict__ meta) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = meta[0] + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bound;
       i += stride)
    big[i] = ~0ULL;
}

// The higher-degree vertices, sorted as keys degree << 32 | id: their
// positions after the lower degrees, their row starts and their classes.
struct BigClassLoad {
  const uint64_t* k;
  const uint64_t* meta;
  __device__ uint64_t operator()(uint64_t i) const {
    if (i >= meta[0]) return 0;
    return (i == 0 || (k[i] >> 32) != (k[i - 1] >> 32)) ? 1 : 0;
  }
};

struct BigClassApply {
  const uint64_t* k;
  const uint64_t* rowptr;
  const uint64_t* meta;
  uint64_t cap;
  IndexView ix;
  __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t first) const {
    const uint64_t nbig = meta[0];
    if (i >= nbig) return;
    const uint64_t x = k[i];
    const uint64_t pos = meta[1] + i;
    ix.vlist[pos] = (uint32_t)x;
    ix.vrow[pos] = rowptr[(uint32_t)x];
    const uint64_t cls = meta[2] + prefix;
    if (first) {
      if (cls < cap) {
        ix.cls_deg[cls] = (uint32_t)(x >> 32);
        ix.cls_start[cls] = (uint32_t)pos;
      } else {
        atomicAdd((unsigned long long*)&ix.hdr->overflow, 1ULL);
      }
    }
    if (i == nbig - 1) {
      const uint64_t c = cls + first;
      ix.hdr->num_classes = (uint32_t)(c < cap ? c : cap);
    }
  }
};

struct ClassLoad {
  const uint64_t* k;
  __device__ uint64_t operator()(uint64_t i) const {
    return (i == 0 || (k[i] >> 32) != (k[i - 1] >> 32)) ? 1 : 0;
  }
};

struct ClassApply {
  const uint64_t* k;
  const uint64_t* rowptr;
  uint64_t N;
  uint64_t cap;
  uint64_t dmask;
  IndexView ix;
  __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t first) const {
    const uint64_t x = k[i];
    ix.vlist[i] = (uint32_t)x;
    ix.vrow[i] = rowptr[(uint32_t)x];
    if (first) {
      if (prefix < cap) {
        ix.cls_deg[prefix] = (uint32_t)((x >> 32) & dmask);
        ix.cls_start[prefix] = (uint32_t)i;
      } else {
        atomicAdd((unsigned long long*)&ix.hdr->overflow, 1ULL);
      }
    }
    if (i == N - 1) {
      const uint64_t c = prefix + first;
      ix.hdr->num_classes = (uint32_t)(c < cap ? c : cap);
    }
  }
};

// wedges of class j: (vertices in the class) * C(d_j, 2)
__device__ inline uint64_t class_wedges(const IndexView& ix, uint64_t n, uint32_t C, uint64_t j) {
  const uint64_t d = ix.cls_deg[j];
  const uint64_t end = (j + 1 < C) ? ix.cls_start[j + 1] : n;
  const uint64_t cnt = end - ix.cls_start[j];
  return d < 2 ? 0 : cnt * (d * (d - 1) / 2);
}

struct WedgeLoad {
  IndexView ix;
  uint64_t n;
  __device__ uint64_t operator()(uint64_t j) const {
    const uint32_t C = ix.hdr->num_classes;
    return j < C ? class_wedges(ix, n, C, j) : 0;
  }
};

struct CumwApply {
  IndexView ix;
  __device__ void operator()(uint64_t j, uint64_t prefix, uint64_t w) const {
    if (j < ix.hdr->num_classes) ix.cls_cumw[j] = prefix + w;
  }
};

// Slot of (graph g, bin b) in the fill table: G * (max_bins + 1) slots,
// slot b = max_bins of a graph standing for "bins >= max_bins".
__device__ inline uint64_t slot_of(uint32_t g, uint32_t b, uint32_t max_bins) {
  return (uint64_t)g * (max_bins + 1) + b;
}

// One thread per class: add its vertices and wedges to its (graph, bin), and
// record the first class of every slot it starts: first_cls[s] = first
// class whose slot is >= s.
__global__ void k_bin_accumulate(IndexView ix, uint64_t n, uint32_t tau, uint64_t omega,
                                 uint32_t max_bins, const uint32_t* __restrict__ voff, uint32_t G,
                                 uint64_t* __restrict__ n_b, uint64_t* __restrict__ p_b,
                                 uint32_t* __restrict__ first_cls) {
  const uint32_t C = ix.hdr->num_classes;
  const uint64_t nslots = (uint64_t)G * (max_bins + 1);
  uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; j < C; j += stride) {
    const uint64_t d = ix.cls_deg[j];
    const uint64_t end = (j + 1 < C) ? ix.cls_start[j + 1] : n;
    const uint64_t cnt = end - ix.cls_start[j];
    const uint32_t g = graph_of(voff, G, ix.vlist[ix.cls_start[j]]);
    const uint32_t b = d == 0 ? 0 : bin_id_capped(d, tau, omega, max_bins);
    if (d > 0) {
      if (b >= max_bins) {
        atomicAdd((unsigned long long*)&ix.hdr->overflow, (unsigned long long)cnt);
      } else {
        atomicAdd((unsigned long long*)&n_b[(uint64_t)g * max_bins + b], (unsigned long long)cnt);
        atomicAdd((unsigned long long*)&p_b[(uint64_t)g * max_bins + b],
                  (unsigned long long)class_wedges(ix, n, C, j));
      }
    }
    const uint64_t s = slot_of(g, b, max_bins);
    int64_t sprev = -1;
    if (j > 0) {
      const uint64_t dp = ix.cls_deg[j - 1];
      const uint32_t gp = graph_of(voff, G, ix.vlist[ix.cls_start[j - 1]]);
      sprev = (int64_t)slot_of(gp, dp == 0 ? 0 : bin_id_capped(dp, tau, omega, max_bins), max_bins);
    }
    for (int64_t t = sprev + 1; t <= (int64_t)s; ++t) first_cls[t] = (uint32_t)j;
    if (j == C - 1)
      for (uint64_t t = s + 1; t <= nslots; ++t) first_cls[t] = C;
  }
}

// One thread per (graph, row): rows b < max_bins are the bins, row max_bins
// the graph's global stream (every vertex of the graph with d >= 2).
__global__ void k_bin_finalize(IndexView ix, uint64_t n, uint64_t cap, uint32_t tau,
                               uint64_t omega, uint32_t max_bins, uint32_t G,
                               const uint64_t* __restrict__ n_b, const uint64_t* __restrict__ p_b,
                               const uint32_t* __restrict__ first_cls) {
  const uint64_t f = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t rows = (uint64_t)G * (max_bins + 1);
  if (f >= rows) return;
  const uint32_t g = (uint32_t)(f / (max_bins + 1));
  const uint32_t b = (uint32_t)(f % (max_bins + 1));
  BinMeta mt;
  mt.pad[0] = mt.pad[1] = 0;
  if (b < max_bins) {
    mt.lo_deg = bin_lo_deg(b, tau, omega);
    mt.hi_deg = bin_lo_deg(b + 1, tau, omega);
    mt.n_b = n_b[(uint64_t)g * max_bins + b];
    mt.p_b = p_b[(uint64_t)g * max_bins + b];
    mt.cls_lo = first_cls[slot_of(g, b, max_bins)];
    mt.cls_hi = first_cls[slot_of(g, b + 1, max_bins)];
    mt.cumw_base = mt.cls_lo > 0 ? ix.cls_cumw[mt.cls_lo - 1] : 0;
  } else {
    mt.lo_deg = 2;
    mt.hi_deg = ~0ULL;
    mt.n_b = 0;
    mt.cls_lo = first_cls[slot_of(g, 0, max_bins)];
    mt.cls_hi = first_cls[slot_of(g + 1, 0, max_bins)];
    mt.cumw_base = mt.cls_lo > 0 ? ix.cls_cumw[mt.cls_lo - 1] : 0;
    const uint64_t top = mt.cls_hi > 0 ? ix.cls_cumw[mt.cls_hi - 1] : 0;
    mt.p_b = mt.cls_hi > mt.cls_lo ? top - mt.cumw_base : 0;
  }
  ix.bins[f] = mt;
  if (f == 0) {
    ix.hdr->n = (uint32_t)n;
    ix.hdr->max_bins = max_bins;
    ix.hdr->tau = tau;
    ix.hdr->omega = omega;
    ix.hdr->class_cap = cap;
    ix.hdr->num_graphs = G;
  }
}

struct BinsWorkspace {
  uint64_t* keys_a;
  uint64_t* keys_b;
  uint64_t* scan_ws;
  uint32_t* first_cls;
  uint64_t* meta;  // one graph: [0] vertices of degree >= kRowsDirect, [1] their first
                   // position, [2] classes of lower degree, [3] 1 if the pass by
                   // degree gave up waiting between tiles
  void* radix;
};

static size_t bins_layout(uint64_t n, uint32_t G, uint32_t max_bins, BinsWorkspace* w,
                          void* base) {
  char* c = (char*)base;
  size_t off = 0;
  const size_t keys = round_up((size_t)(n ? n : 1) * 8, 256);
  if (w) w->keys_a = (uint64_t*)(c + off);
  off += keys;
  if (w) w->keys_b = (uint64_t*)(c + off);
  off += keys;
  if (w) w->scan_ws = (uint64_t*)(c + off);
  off += round_up(scan_ws_elems(n + 1) * 8, 256);
  if (w) w->first_cls = (uint32_t*)(c + off);
  off += round_up(4 * ((size_t)G * ((size_t)max_bins + 1) + 2), 256);
  if (w) w->meta = (uint64_t*)(c + off);
  off += 256;
  if (w) w->radix = (void*)(c + off);
  off += os_scratch_bytes(n);
  return off;
}

size_t bins_workspace_bytes(uint64_t n_total, uint32_t G, uint32_t max_bins) {
  return bins_layout(n_total, G, max_bins, nullptr, nullptr);
}

int bins_build(const uint64_t* d_rowptr, uint64_t n, uint64_t m_total, const uint32_t* d_voff,
               uint32_t G, uint32_t max_n, uint32_t tau, uint64_t omega, uint32_t max_bins,
               uint64_t* d_n_b, uint64_t* d_p_b, void* d_index, void* d_workspace,
               hipStream_t st) {
  BinsWorkspace w;
  bins_layout(n, G, max_bins, &w, d_workspace);
  IndexView ix = index_view(d_index, n, m_total, G, max_bins);
  const uint64_t cap = class_capacity(n, m_total, G);
  const int gbits = G > 1 ? bit_width((uint64_t)G - 1) : 0;
  const int gshift = 64 - gbits;
  const uint64_t dmask = (gbits > 0) ? ((1ULL << (32 - gbits)) - 1) : 0xFFFFFFFFULL;
  int rc;
  if ((rc = fill<uint64_t>((uint64_t*)ix.hdr, sizeof(IndexHeader) / 8, 0, st))) return rc;
  if ((rc = fill<uint64_t>(d_n_b, (uint64_t)G * max_bins, 0, st))) return rc;
  if ((rc = fill<uint64_t>(d_p_b, (uint64_t)G * max_bins, 0, st))) return rc;
  uint64_t dbound = (uint64_t)(max_n ? max_n : 1) - 1;
  if (m_total < dbound) dbound = m_total;
  const OsScratch osc = os_scratch(w.radix, n);
  if (G == 1 && n > 0) {
    if ((rc = fill<uint64_t>(osc.hist, 256, 0, st))) return rc;
    {
      // few enough workgroups that their global adds (one per nonzero
      // counter) do not queue on the 256 counters
      uint64_t blocks = ceil_div(n, 256);
      if (blocks > 2048) blocks = 2048;
      k_deg_hist<<<(unsigned)blocks, 256, 0, st>>>(d_rowptr, (uint32_t)n, ix.vcode, ix.vmeta,
                                                   osc.hist);
      WEDGE_LAUNCH_CHECK("k_deg_hist");
    }
    if ((rc = onesweep_rows(RowSink{d_rowptr, ix.vlist, ix.vrow, w.keys_a}, n, osc, st)))
      return rc;
    // the sort below clears the stall count: keep this pass's in meta[3]
    if ((rc = fill<uint64_t>(w.meta + 3, 1, 0, st))) return rc;
    if ((rc = os_flag_stalls(osc, w.meta + 3, 1, st))) return rc;
    k_rows_classes<<<1, 256, 0, st>>>(osc.hist, osc.base, cap, ix, w.meta);
    WEDGE_LAUNCH_CHECK("k_rows_classes");
    // vertices of degree >= kRowsDirect: at most 2m / kRowsDirect of them
    uint64_t bound = 2 * m_total / kRowsDirect;
    if (bound > n) bound = n;
    if (bound > 0) {
      {
        uint64_t blocks = ceil_div(bound, 256);
        if (blocks > 4096) blocks = 4096;
        k_rows_tail<<<(unsigned)blocks, 256, 0, st>>>(w.keys_a, bound, w.meta);
        WEDGE_LAUNCH_CHECK("k_rows_tail");
      }
      int shifts[16];
      int np = 0;
      for (int s = 0; s < bit_width(dbound); s += 8) shifts[np++] = 32 + s;
      uint64_t* sorted = nullptr;
      rc = onesweep_sort_keys(w.keys_a, w.keys_b, bound, shifts, np, osc, st, &sorted);
      if (rc) return rc;
      rc = scan_apply<uint64_t>(BigClassLoad{sorted, w.meta},
                                BigClassApply{sorted, d_rowptr, w.meta, cap, ix}, bound,
                                w.scan_ws, st);
      if (rc) return rc;
    }
  } else {
    {
      uint64_t blocks = ceil_div(n, 256);
      if (blocks > 65536) blocks = 65536;
      k_deg_keys<<<(unsigned)blocks, 256, 0, st>>>(d_rowptr, (uint32_t)n, d_voff, G, gshift,
                                                   dmask, w.keys_a, ix.vcode, ix.vmeta);
      WEDGE_LAUNCH_CHECK("k_deg_keys");
    }
    // sort by the degree digits, then by the graph digits; ids stay ascending
    int shifts[16];
    int np = 0;
    for (int s = 0; s < bit_width(dbound); s += 8) shifts[np++] = 32 + s;
    for (int s = 0; s < gbits; s += 8) shifts[np++] = gshift + s;
    uint64_t* sorted = nullptr;
    rc = onesweep_sort_keys(w.keys_a, w.keys_b, n, shifts, np, osc, st, &sorted);
    if (rc) return rc;
    rc = scan_apply<uint64_t>(ClassLoad{sorted}, ClassApply{sorted, d_rowptr, n, cap, dmask, ix},
                              n, w.scan_ws, st);
    if (rc) return rc;
  }
  rc = scan_apply<uint64_t>(WedgeLoad{ix, n}, CumwApply{ix}, cap, w.scan_ws, st);
  if (rc) return rc;
  {
    uint64_t blocks = ceil_div(cap, 256);
    if (blocks > 4096) blocks = 4096;
    k_bin_accumulate<<<(unsigned)blocks, 256, 0, st>>>(ix, n, tau, omega, max_bins, d_voff, G,
                                                       d_n_b, d_p_b, w.first_cls);
    WEDGE_LAUNCH_CHECK("k_bin_accumulate");
  }
  const uint64_t rows = (uint64_t)G * (max_bins + 1);
  k_bin_finalize<<<(unsigned)ceil_div(rows, 256), 256, 0, st>>>(ix, n, cap, tau, omega, max_bins,
                                                                G, d_n_b, d_p_b, w.first_cls);
  WEDGE_LAUNCH_CHECK("k_bin_finalize");
  // a sort whose bounded wait gave up leaves overflow = 2^64 - 1
  if (G == 1 && n > 0) {
    k_flag_if_set<<<1, 64, 0, st>>>(w.meta + 3, (uint64_t*)&ix.hdr->overflow, ~0ULL);
    WEDGE_LAUNCH_CHECK("k_flag_if_set");
  }
  return os_flag_stalls(osc, (uint64_t*)&ix.hdr->overflow, ~0ULL, st);
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_index_bytes(uint32_t n, uint64_t m, uint32_t max_bins) {
  return index_bytes(n, m, 1, max_bins);
}

extern "C" size_t wedge_bin_counts_workspace(uint32_t n) {
  return bins_workspace_bytes(n, 1, 4096);
}

extern "C" int wedge_bin_counts(const uint64_t* d_rowptr, uint32_t n, uint64_t m, uint32_t tau,
                                uint64_t omega, uint32_t max_bins, uint64_t* d_n_b,
                                uint64_t* d_p_b, void* d_index, size_t index_bytes_given,
                                void* d_workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_bin_counts: n must be >= 1");
  if (tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_bin_counts: need tau >= 1 and integer omega >= 2");
  if (max_bins == 0 || max_bins > 4096)
    return set_error(WEDGE_ERANGE, "wedge_bin_counts: max_bins must be in [1, 4096]");
  if (!d_rowptr || !d_n_b || !d_p_b || !d_index || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_bin_counts: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_n_b, 8) || !aligned(d_p_b, 8) ||
      !aligned(d_index, 256) || !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_bin_counts: misaligned pointer");
  if (index_bytes_given < index_bytes(n, m, 1, max_bins))
    return set_error(WEDGE_EWORKSPACE, "wedge_bin_counts: index %zu < %zu bytes",
                     index_bytes_given, index_bytes(n, m, 1, max_bins));
  if (workspace_bytes < wedge_bin_counts_workspace(n))
    return set_error(WEDGE_EWORKSPACE, "wedge_bin_counts: workspace %zu < %zu bytes",
                     workspace_bytes, wedge_bin_counts_workspace(n));
  return bins_build(d_rowptr, n, m, nullptr, 1, n, tau, omega, max_bins, d_n_b, d_p_b, d_index,
                    d_workspace, (hipStream_t)stream);
}

extern "C" int wedge_index_status(const void* d_index, uint32_t* h_num_classes,
                                  uint64_t* h_overflow, uint64_t* h_empty_bin_samples,
                                  uint64_t* h_mismatch, void* stream) {
  clear_error();
  if (!d_index || !aligned(d_index, 256))
    return set_error(WEDGE_EINVAL, "wedge_index_status: null or misaligned index");
  IndexHeader h;
  WEDGE_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  WEDGE_HIP_TRY(hipMemcpy(&h, d_index, sizeof(h), hipMemcpyDeviceToHost));
  if (h_num_classes) *h_num_classes = h.num_classes;
  if (h_overflow) *h_overflow = h.overflow;
  if (h_empty_bin_samples) *h_empty_bin_samples = h.empty_bin_samples;
  if (h_mismatch) *h_mismatch = h.mismatch;
  return WEDGE_OK;
}
