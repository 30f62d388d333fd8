// wedge_sample_close: uniform wedge samples per degree bin and exact closure
// tests (Thm. cd-est / td-est; centre-then-pair construction of Sec. 3.2;
// pair law of the Sampling procedure of Alg. phase2c; exact edge match of
// Alg. phase3b; classes q0..q3 of Alg. phase4c).
//
// Work layout: a workgroup takes one tile of consecutive sample indices of
// one (graph, bin) row.  It stages the row's cumulative-wedge table (one
// entry per distinct degree, or every S-th entry when the row has more than
// the LDS holds) in LDS, then each lane carries U independent samples
// through the dependent gather chain
//     Philox -> centre class (LDS search) -> adjacency start of the centre
//            -> col (a, c) -> row-start word of a (and of c when a's row
//            is long) -> search in the chosen row,
// issuing the loads of its U samples back to back so that U x (waves per CU)
// chains are in flight per CU.  Class counts are reduced per wave with
// shuffles, per workgroup in LDS, and added to the row's four uint64
// counters with one atomic each: integer sums, so the result does not depend
// on tiling or scheduling.
//
// Two launch forms share the tile routine: a grid of tiles with the task
// table in the kernel arguments (one graph), and a persistent grid that
// pulls tiles of every (graph, bin) row of a batch from a device work queue.
#include "common.hpp"
#include "rng.hpp"
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "hash.hpp"
#include "sample.hpp"
#include "scan.hpp"

namespace wedge {

// Degree code (floor of 8 log2 of the degree, Mitchell's form) above which
// the closure step also reads the other endpoint's word to search the
// shorter row: about degree 4,500.
constexpr uint64_t kLongRowCode = 96;
// No vertex word has every bit set (row starts are below 2^41).
constexpr uint64_t kNoWord = ~0ULL;

constexpr int kLdsClasses = 1024;
constexpr uint32_t kGlobalWord = 0xFFFFFFFFu;

struct TileSmem {
  uint64_t cumw[kLdsClasses];
  uint32_t deg[kLdsClasses];
  uint32_t start[kLdsClasses];
  unsigned long long red[5];
  uint64_t item[2];
  uint64_t arange[2];  // allocation form: the tile's first and last vertex
};

// The row's cumulative-wedge table in LDS: one entry per class, or the last
// class of every group of S when the row has more classes than LDS holds.
struct StagedRow {
  uint32_t S, ngroups, ncls;
};

__device__ inline StagedRow stage_row(const SamplerCtx& A, TileSmem& sm, const BinMeta& M) {
  StagedRow R;
  R.ncls = M.cls_hi - M.cls_lo;
  R.S = (R.ncls + kLdsClasses - 1) / kLdsClasses;  // classes per staged group
  R.ngroups = (R.ncls + R.S - 1) / R.S;
  for (uint32_t i = threadIdx.x; i < R.ngroups; i += kSampWG) {
    const uint32_t last = min((i + 1) * R.S, R.ncls) - 1;
    sm.cumw[i] = A.ix.cls_cumw[M.cls_lo + last];
    if (R.S == 1) {
      sm.deg[i] = A.ix.cls_deg[M.cls_lo + i];
      sm.start[i] = A.ix.cls_start[M.cls_lo + i];
    }
  }
  return R;
}

// Centre of wedge index W of the row: the first staged group whose
// cumulative count exceeds W, then (when groups hold several classes) the
// class inside; the centre is the (W - wedges before the class) / C(d, 2)-th
// vertex of the class.
__device__ inline void centre_of(const SamplerCtx& A, const TileSmem& sm, const BinMeta& M,
                                 const StagedRow& R, uint64_t W, uint64_t* d, uint64_t* vi) {
  uint32_t l = 0, h = R.ngroups;
  while (l < h) {
    const uint32_t mid = (l + h) >> 1;
    if (sm.cumw[mid] > W) h = mid; else l = mid + 1;
  }
  uint64_t dd, st, cprev;
  if (R.S == 1) {
    dd = sm.deg[l];
    st = sm.start[l];
    cprev = l > 0 ? sm.cumw[l - 1] : M.cumw_base;
  } else {
    uint32_t jl = l * R.S, jh = min((l + 1) * R.S, R.ncls);
    while (jl < jh) {
      const uint32_t mid = (jl + jh) >> 1;
      if (A.ix.cls_cumw[M.cls_lo + mid] > W) jh = mid; else jl = mid + 1;
    }
    const uint64_t j = (uint64_t)M.cls_lo + jl;
    dd = A.ix.cls_deg[j];
    st = A.ix.cls_start[j];
    cprev = j > 0 ? A.ix.cls_cumw[j - 1] : 0;
  }
  *d = dd;
  uint64_t v = st + (W - cprev) / (dd * (dd - 1) / 2);
  if (v >= A.n) v = A.n - 1;  // unreachable for a consistent index
  *vi = v;
}

// Allocation form: the row position i in [lo, hi) of the vertex holding
// sample s, i.e. the last i with pre[off + i] <= pre[off] + s.
__device__ inline uint64_t alloc_vertex(const SamplerCtx& A, const AllocRow& R, uint64_t s,
                                        uint64_t lo, uint64_t hi) {
  const uint64_t g = A.alloc_pre[R.off] + s;
  while (hi - lo > 1) {
    const uint64_t mid = (lo + hi) >> 1;
    if (A.alloc_pre[R.off + mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// One tile: samples [s0, s1) of index row f (graph g, bin word bword).
// kDraw: stop after the draws and record (centre, i, j) (streamed path).
template <int U, bool kAlloc = false, bool kDraw = false>
__device__ void sample_tile(const SamplerCtx& A, TileSmem& sm, uint64_t f, uint32_t bword,
                            uint64_t gword, uint64_t s0, uint64_t s1, uint64_t fslot,
                            uint64_t sbase) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const BinMeta M = A.ix.bins[f];
  if (M.p_b == 0) {
    if (tid == 0) atomicAdd((unsigned long long*)&A.ix.hdr->empty_bin_samples, s1 - s0);
    return;
  }
  const bool global = (bword == kGlobalWord);
  const StagedRow R = stage_row(A, sm, M);
  if (tid < 5) sm.red[tid] = 0;
  AllocRow AR{0, 0, 0, 0};
  if (kAlloc) {
    AR = A.alloc[f];
    if (tid < 2) sm.arange[tid] = alloc_vertex(A, AR, tid == 0 ? s0 : s1 - 1, 0, AR.count);
  }
  __syncthreads();

  const uint64_t seed = A.seed;
  const uint64_t bw = bword;
  const uint32_t* __restrict__ col = A.col;
  uint32_t cnt0 = 0, cnt1 = 0, cnt2 = 0, cnt3 = 0;
  uint64_t probes = 0;

  for (uint64_t base = s0; base < s1; base += (uint64_t)kSampWG * U) {
    uint64_t s[U], W[U], x1[U], d[U], vi[U], rp[U], lo[U], len[U];
    uint32_t v[U], a[U], c[U], key[U];
    uint64_t ia[U], ic[U];
    bool act[U], found[U];
    // 1. random words and the centre's wedge index
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s[u] = base + (uint64_t)u * kSampWG + tid;
      act[u] = s[u] < s1;
      W[u] = 0;
      x1[u] = 0;
      if (act[u]) {
        const U64x4 o = philox4x64_10(s[u], bw, gword, 0, seed, A.domain);
        if (!kAlloc)
          W[u] = M.cumw_base + below_from(o.w[0], M.p_b, seed, A.domain, s[u], bw, gword, 0);
        x1[u] = o.w[1];
      }
    }
    // 2. the centre: class by the staged table, then the vertex (allocation
    //    form: the vertex whose share of the row's samples holds s)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t dd = 2, vv = 0;
      if (act[u]) {
        if (kAlloc) {
          vv = AR.pos_lo + alloc_vertex(A, AR, s[u], sm.arange[0], sm.arange[1] + 1);
          const uint32_t x = A.ix.vlist[vv];
          dd = A.rowptr[x + 1] - A.rowptr[x];
        } else {
          centre_of(A, sm, M, R, W[u], &dd, &vv);
        }
      }
      d[u] = dd;
      vi[u] = vv;
    }
    // the centre's adjacency start comes straight from the index; its id is
    // only needed for a dump
#pragma unroll
    for (int u = 0; u < U; ++u) rp[u] = act[u] ? A.ix.vrow[vi[u]] : 0;
    if (A.dump) {
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = act[u] ? A.ix.vlist[vi[u]] : 0;
    }
    // 3. ordered pair of distinct neighbours, numbered in ascending id order
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ia[u] = ic[u] = 0;
      if (act[u]) {
        const uint64_t dm1 = d[u] - 1;
        const uint64_t o = below_from(x1[u], d[u] * dm1, seed, A.domain, s[u], bw, gword, 1);
        const uint64_t i = o / dm1;
        const uint64_t r = o - i * dm1;
        ia[u] = i;
        ic[u] = r + (r >= i ? 1 : 0);
      }
    }
    if (kDraw) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (act[u] && s[u] - sbase < A.dump_per_bin) {
          wedge_sample_rec rec;
          rec.v = v[u];
          rec.a = (uint32_t)ia[u];
          rec.c = (uint32_t)ic[u];
          rec.cls = 0;
          A.dump[f * A.dump_per_bin + (s[u] - sbase)] = rec;
        }
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = act[u] ? col[rp[u] + ia[u]] : 0;
      c[u] = act[u] ? col[rp[u] + ic[u]] : 0;
    }
    // 4. closure: search one endpoint in the row of the other.  One 8-byte
    //    word per vertex holds its row start and, in the top byte, its degree
    //    code.  The search takes a's row unless that row is long (code above
    //    kLongRowCode); then c's word is read too and the row with the
    //    smaller code is searched (tie: a's).  A random line costs more than
    //    the extra probes of a short row, so c's word is read only where the
    //    search it may save is long.
    uint64_t da[U], dc[U], my[U];
    bool in_a[U];
    if (A.hash) {
      // closure by lookup in the edge table; the endpoints' degrees are read
      // only where a class or a record needs them
#pragma unroll
      for (int u = 0; u < U; ++u) {
        found[u] = act[u] && A.closure && hash_has_edge(A.hash, A.hash_bits, a[u], c[u], &probes);
        da[u] = dc[u] = 0;
        if (act[u] && (A.feat || (found[u] && !global))) {
          da[u] = (A.ix.vmeta[a[u] + 1] & kRowMask) - (A.ix.vmeta[a[u]] & kRowMask);
          dc[u] = (A.ix.vmeta[c[u] + 1] & kRowMask) - (A.ix.vmeta[c[u]] & kRowMask);
        }
      }
    } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      uint64_t ma = 0, mc = 0;
      if (act[u]) ma = A.ix.vmeta[a[u]];
      const bool both = act[u] && (ma >> 56) > kLongRowCode;
      if (both) mc = A.ix.vmeta[c[u]];
      in_a[u] = !both || (ma >> 56) <= (mc >> 56);
      const uint32_t x = in_a[u] ? a[u] : c[u];
      // the other endpoint's word, or kNoWord when it has not been read
      my[u] = in_a[u] ? (both ? mc : kNoWord) : ma;
      uint64_t r0 = 0, r1 = 0;
      if (act[u]) {
        r0 = (in_a[u] ? ma : mc) & kRowMask;
        r1 = A.ix.vmeta[x + 1] & kRowMask;
      }
      const uint64_t dx = r1 - r0;
      da[u] = in_a[u] ? dx : 0;
      dc[u] = in_a[u] ? 0 : dx;
      lo[u] = r0;
      len[u] = (act[u] && A.closure) ? dx : 0;
      key[u] = in_a[u] ? c[u] : a[u];
      found[u] = false;
    }
    // Search [lo, lo + len) for key.  Ids are spread over [0, n) and a row
    // holds them in ascending order, so in a row of more than 16 entries of a
    // single graph the first probe goes where the key's share of the id range
    // points; the next ones gallop away from it on the key's side (2, 4, 8,
    // ... entries past the last probe) until one passes the key, and a
    // bisection finishes inside that step.  The key is usually a few entries
    // from the guess, so most searches stay in the guess's cache line, and a
    // bad guess costs O(log distance) probes.  Stage 0: interpolated probe;
    // 1: galloping; 2: bisection.
    const float inv_n = 1.0f / (float)A.n;  // the guess needs no precision
    uint32_t stage[U];
    uint64_t win[U];
    bool right[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool interp = A.num_graphs == 1 && len[u] > 16;
      stage[u] = interp ? 0 : 2;
      win[u] = interp ? 2 : 0;  // first galloping step
      right[u] = true;
    }
    bool more = true;
    while (more) {
      uint32_t x[U];
      uint64_t h[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (len[u] == 0) continue;
        if (stage[u] == 0) {
          h[u] = (uint64_t)((float)len[u] * ((float)key[u] * inv_n));
        } else if (stage[u] == 1) {
          // the key is past the last probe: one step further on that side
          if (right[u])
            h[u] = win[u] < len[u] ? win[u] : len[u] - 1;
          else
            h[u] = len[u] > win[u] ? len[u] - 1 - win[u] : 0;
        } else {
          h[u] = len[u] >> 1;
        }
        if (h[u] >= len[u]) h[u] = len[u] - 1;
        x[u] = col[lo[u] + h[u]];
      }
      more = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (len[u] > 0) {
          ++probes;
          // a galloping probe with the key still beyond it doubles the step
          bool again = false;
          if (x[u] == key[u]) {
            found[u] = true;
            len[u] = 0;
          } else if (x[u] < key[u]) {
            lo[u] += h[u] + 1;
            len[u] -= h[u] + 1;
            again = stage[u] == 1 && right[u];
            right[u] = true;
          } else {
            len[u] = h[u];
            again = stage[u] == 1 && !right[u];
            right[u] = false;
          }
          if (again)
            win[u] *= 2;
          else
            stage[u] = stage[u] < 2 ? stage[u] + 1 : 2;
          more |= len[u] > 0;
        }
      }
    }
    // the other endpoint's degree: for the class of a closed bin sample, and
    // for every feature record
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (act[u] && (A.feat || (found[u] && !global))) {
        const uint32_t y = in_a[u] ? c[u] : a[u];
        const uint64_t wy = my[u] == kNoWord ? A.ix.vmeta[y] : my[u];
        const uint64_t dy = (A.ix.vmeta[y + 1] & kRowMask) - (wy & kRowMask);
        if (in_a[u]) dc[u] = dy; else da[u] = dy;
      }
    }
    }  // search form
    // 5. class and tallies
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!act[u]) continue;
      uint32_t cls = 0;
      if (found[u]) {
        cls = global ? 3u
                     : 1u + (M.lo_deg <= da[u] && da[u] < M.hi_deg ? 1u : 0u) +
                           (M.lo_deg <= dc[u] && dc[u] < M.hi_deg ? 1u : 0u);
      }
      cnt0 += cls == 0;
      cnt1 += cls == 1;
      cnt2 += cls == 2;
      cnt3 += cls == 3;
      if (A.dump && s[u] - sbase < A.dump_per_bin) {
        wedge_sample_rec rec;
        rec.v = v[u];
        rec.a = a[u];
        rec.c = c[u];
        rec.cls = cls;
        A.dump[f * A.dump_per_bin + (s[u] - sbase)] = rec;
      }
      if (A.feat) {
        wedge_feature_rec fr;
        fr.dv = (uint32_t)d[u];
        fr.dlo = (uint32_t)min(da[u], dc[u]);
        fr.dhi = (uint32_t)max(da[u], dc[u]);
        fr.bin = (uint16_t)bin_id_capped(d[u], A.tau, A.omega, A.max_bins);
        fr.closed = found[u] ? 1 : 0;
        fr.cls = (uint8_t)cls;
        A.feat[fslot * A.feat_stride + (s[u] - sbase)] = fr;
      }
    }
  }
  unsigned long long r0 = wave_sum<unsigned long long>(cnt0);
  unsigned long long r1 = wave_sum<unsigned long long>(cnt1);
  unsigned long long r2 = wave_sum<unsigned long long>(cnt2);
  unsigned long long r3 = wave_sum<unsigned long long>(cnt3);
  unsigned long long r4 = wave_sum<unsigned long long>(probes);
  if (lane == 0) {
    atomicAdd(&sm.red[0], r0);
    atomicAdd(&sm.red[1], r1);
    atomicAdd(&sm.red[2], r2);
    atomicAdd(&sm.red[3], r3);
    atomicAdd(&sm.red[4], r4);
  }
  __syncthreads();
  if (tid < 4) {
    if (A.q && sm.red[tid]) atomicAdd((unsigned long long*)&A.q[f * 4 + tid], sm.red[tid]);
  } else if (tid == 4 && A.probe_loads) {
    atomicAdd((unsigned long long*)A.probe_loads, sm.red[4]);
  }
  __syncthreads();  // the shared table and tallies are reused by the next tile
}

__device__ inline bool header_ok(const SamplerCtx& A) {
  const IndexHeader* H = A.ix.hdr;
  return H->n == A.n && H->max_bins == A.max_bins && H->class_cap == A.class_cap &&
         H->num_graphs == A.num_graphs;
}

template <int U, bool kAlloc = false, bool kDraw = false>
__global__ __launch_bounds__(kSampWG, U == 1 ? 8 : 1) void k_sample_close(const SamplerCtx A, const TaskTable T) {
  __shared__ TileSmem sm;
  const uint64_t tile = blockIdx.x;
  int e = 0;
  for (int i = 1; i < (int)T.ntask; ++i)
    if (T.task[i].tile_begin <= tile) e = i;
  const uint64_t sbase = T.task[e].s_begin;
  const uint64_t s0 = sbase + (tile - T.task[e].tile_begin) * A.spt;
  const uint64_t s1 = min(s0 + A.spt, sbase + T.task[e].k);
  if (s0 >= s1) return;
  if (!header_ok(A)) {
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)&A.ix.hdr->mismatch, 1ULL);
    return;
  }
  sample_tile<U, kAlloc, kDraw>(A, sm, T.task[e].row, T.task[e].bword, T.graph_word, s0, s1,
                                T.task[e].slot, sbase);
}

// Persistent form: tiles of all (graph, row) pairs of a batch come from a
// ticket counter; tile_begin[f] is the exclusive prefix of the tile counts
// of rows f (tile_begin[nrows] = total).  Every workgroup leaves the loop
// once the ticket passes the total.
template <int U>
__global__ __launch_bounds__(kSampWG, U == 1 ? 8 : 1) void k_sample_persistent(const SamplerCtx A,
                                                               const uint64_t* __restrict__ task_k,
                                                               const uint64_t* __restrict__ tile_begin,
                                                               uint64_t nrows,
                                                               unsigned long long* ticket) {
  __shared__ TileSmem sm;
  if (!header_ok(A)) {
    if (threadIdx.x == 0) atomicAdd((unsigned long long*)&A.ix.hdr->mismatch, 1ULL);
    return;
  }
  const uint64_t total = tile_begin[nrows];
  const uint32_t rows_per_graph = A.max_bins + 1;
  for (;;) {
    if (threadIdx.x == 0) {
      const uint64_t t = atomicAdd(ticket, 1ULL);
      uint64_t f = 0;
      if (t < total) {
        uint64_t lo = 0, hi = nrows;  // last f with tile_begin[f] <= t
        while (hi - lo > 1) {
          const uint64_t mid = (lo + hi) >> 1;
          if (tile_begin[mid] <= t) lo = mid; else hi = mid;
        }
        f = lo;
      }
      sm.item[0] = t;
      sm.item[1] = f;
    }
    __syncthreads();
    const uint64_t t = sm.item[0];
    const uint64_t f = sm.item[1];
    __syncthreads();
    if (t >= total) break;
    const uint64_t s0 = A.s_begin + (t - tile_begin[f]) * A.spt;
    const uint64_t s1 = min(s0 + A.spt, A.s_begin + task_k[f]);
    if (s0 >= s1) continue;
    const uint32_t g = (uint32_t)(f / rows_per_graph);
    const uint32_t row = (uint32_t)(f % rows_per_graph);
    sample_tile<U>(A, sm, f, row == A.max_bins ? kGlobalWord : row, g, s0, s1, f, A.s_begin);
  }
}

// One sample per lane and one pass per workgroup: the closure search is a
// chain of dependent loads, and the most waves in flight (the fewest
// registers per lane) hide it best; measured on R-MAT scale 24 this beats
// several samples per lane and longer tiles.
// ------------------------------------------------------------ centre means
// Mean of the control-variate network over all wedges of a drawn centre:
// centre v is drawn with probability p_v / p_row exactly as a sample's
// centre (word 0 of the draw's Philox block), and
//   gbar(v) = (1 / C(d_v, 2)) sum over neighbour pairs {a, c} of
//             G[key(v)][K(d_lo), K(d_hi)],
// with G the network's output for every (key, bucket pair) and K(d) the
// degree bucket (the index keeps it per vertex).  E[gbar(v)] is the mean of
// g over the row's wedges, so these draws estimate the control variate's
// mean without any closure test.  Centres up to kCentreLaneDeg neighbours
// are done by one lane each; larger ones are queued for a wave each.
constexpr uint32_t kCentreLaneDeg = 32;
constexpr uint32_t kCentrePairs = 256 * 257 / 2;

struct CentreArgs {
  const uint32_t* key_of;     // [max_bins][256] key of (bin, centre bucket)
  const float* gtable;        // [keys][kCentrePairs]
  float* out;                 // [rows][stride]
  uint32_t* vout;             // nullable: the drawn centre ids, same layout
  uint64_t stride;
  unsigned long long* queued; // [1] entries in `queue`
  uint64_t* queue;            // [capacity][3]: out index, row start, d << 32 | key
  uint64_t capacity;
};

__device__ inline uint32_t pair_at(uint32_t i, uint32_t j) {  // i <= j
  return j * (j + 1) / 2 + i;
}

template <int Dummy>
__global__ __launch_bounds__(kSampWG) void k_centre_means(const SamplerCtx A, const TaskTable T,
                                                          const CentreArgs C) {
  __shared__ TileSmem sm;
  __shared__ uint8_t s_b[kCentreLaneDeg][kSampWG];
  const int tid = threadIdx.x;
  const uint64_t tile = blockIdx.x;
  int e = 0;
  for (int i = 1; i < (int)T.ntask; ++i)
    if (T.task[i].tile_begin <= tile) e = i;
  const uint64_t sbase = T.task[e].s_begin;
  const uint64_t s0 = sbase + (tile - T.task[e].tile_begin) * A.spt;
  const uint64_t s1 = min(s0 + A.spt, sbase + T.task[e].k);
  if (s0 >= s1) return;
  if (!header_ok(A)) {
    if (tid == 0) atomicAdd((unsigned long long*)&A.ix.hdr->mismatch, 1ULL);
    return;
  }
  const uint32_t f = T.task[e].row;
  const uint64_t bw = T.task[e].bword;
  const BinMeta M = A.ix.bins[f];
  if (M.p_b == 0) {
    if (tid == 0) atomicAdd((unsigned long long*)&A.ix.hdr->empty_bin_samples, s1 - s0);
    return;
  }
  const StagedRow R = stage_row(A, sm, M);
  __syncthreads();
  for (uint64_t s = s0 + tid; s < s1; s += kSampWG) {
    const U64x4 o = philox4x64_10(s, bw, T.graph_word, 0, A.seed, A.domain);
    const uint64_t W =
        M.cumw_base + below_from(o.w[0], M.p_b, A.seed, A.domain, s, bw, T.graph_word, 0);
    uint64_t d, vi;
    centre_of(A, sm, M, R, W, &d, &vi);
    const uint64_t rp = A.ix.vrow[vi];
    const uint64_t idx = T.task[e].slot * C.stride + (s - sbase);
    if (C.vout) C.vout[idx] = A.ix.vlist[vi];
    const uint32_t bin = bw == kGlobalWord ? bin_id_capped(d, A.tau, A.omega, A.max_bins) : f;
    const uint32_t ke = 63 - (uint32_t)__builtin_clzll(d);
    const uint32_t kb = 8 * ke + (uint32_t)(((d - (1ULL << ke)) * 8) >> ke);
    const uint32_t key = bin < A.max_bins ? C.key_of[bin * 256 + (kb < 255 ? kb : 255)]
                                          : 0xFFFFFFFFu;
    if (key == 0xFFFFFFFFu) {  // unreachable for a consistent index and key list
      C.out[idx] = 0.f;
    } else if (d <= kCentreLaneDeg) {
      for (uint32_t x = 0; x < d; ++x) s_b[x][tid] = A.ix.vcode[A.col[rp + x]];
      const float* G = C.gtable + (uint64_t)key * kCentrePairs;
      double acc = 0.0;
      for (uint32_t x = 1; x < d; ++x) {
        const uint32_t bx = s_b[x][tid];
        for (uint32_t y = 0; y < x; ++y) {
          const uint32_t by = s_b[y][tid];
          acc += (double)G[bx < by ? pair_at(bx, by) : pair_at(by, bx)];
        }
      }
      C.out[idx] = (float)(acc / (double)(d * (d - 1) / 2));
    } else {
      const uint64_t at = atomicAdd(C.queued, 1ULL);
      if (at < C.capacity) {
        C.queue[3 * at + 0] = idx;
        C.queue[3 * at + 1] = rp;
        C.queue[3 * at + 2] = (d << 32) | key;
      }
    }
  }
}

// Queued centres, one wave each: bucket histogram of the neighbours, then
// every pair of non-empty buckets with its count.
__global__ __launch_bounds__(256) void k_centre_wide(const SamplerCtx A, const CentreArgs C) {
  __shared__ uint32_t s_h[4][256];
  __shared__ uint16_t s_list[4][256];
  __shared__ uint32_t s_cnt[4][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t total = min((uint64_t)*C.queued, C.capacity);
  const uint64_t nwaves = (uint64_t)gridDim.x * 4;
  for (int i = lane; i < 256; i += 64) s_h[wave][i] = 0;
  __builtin_amdgcn_wave_barrier();
  for (uint64_t q = (uint64_t)blockIdx.x * 4 + wave; q < total; q += nwaves) {
    const uint64_t idx = C.queue[3 * q + 0];
    const uint64_t rp = C.queue[3 * q + 1];
    const uint64_t dk = C.queue[3 * q + 2];
    const uint64_t d = dk >> 32;
    const uint32_t key = (uint32_t)dk;
    for (uint64_t x = lane; x < d; x += 64) atomicAdd(&s_h[wave][A.ix.vcode[A.col[rp + x]]], 1u);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t h[4], nz = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      h[t] = s_h[wave][lane * 4 + t];
      nz += h[t] > 0;
    }
    uint32_t pre = nz;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(pre, off, 64);
      if (lane >= off) pre += y;
    }
    const uint32_t u = __shfl(pre, 63, 64);
    uint32_t at = pre - nz;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (h[t] > 0) {
        s_list[wave][at] = (uint16_t)(lane * 4 + t);
        s_cnt[wave][at] = h[t];
        ++at;
      }
      s_h[wave][lane * 4 + t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float* G = C.gtable + (uint64_t)key * kCentrePairs;
    double acc = 0.0;
    const uint32_t np = u * (u + 1) / 2;
    for (uint32_t t = lane; t < np; t += 64) {
      uint32_t j = (uint32_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
      while (j * (j + 1) / 2 > t) --j;
      while ((j + 1) * (j + 2) / 2 <= t) ++j;
      const uint32_t i = t - j * (j + 1) / 2;
      const uint64_t hi = s_cnt[wave][i], hj = s_cnt[wave][j];
      const uint64_t cnt = (i == j) ? hi * (hi - 1) / 2 : hi * hj;
      if (cnt) acc += (double)cnt * (double)G[pair_at(s_list[wave][i], s_list[wave][j])];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) C.out[idx] = (float)(acc / (double)(d * (d - 1) / 2));
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

SampleTuning default_tuning(uint64_t total) {
  (void)total;
  SampleTuning t;
  t.U = 1;
  t.spt = (uint64_t)kSampWG;
  t.workgroups = 256 * 8;
  return t;
}

void normalise(SampleTuning& t) {
  if (t.U != 1 && t.U != 2 && t.U != 4 && t.U != 8) t.U = 4;
  const uint64_t unit = (uint64_t)kSampWG * t.U;
  if (t.spt < unit) t.spt = unit;
  t.spt = ceil_div(t.spt, unit) * unit;
  if (t.workgroups == 0) t.workgroups = 256 * 8;
}

static int launch_tasks(const SamplerCtx& A, TaskTable& T, int U, hipStream_t st) {
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < T.ntask; ++i) {
    T.task[i].tile_begin = tiles;
    tiles += ceil_div(T.task[i].k, A.spt);
  }
  if (tiles == 0) return WEDGE_OK;
  if (tiles > 0x7FFFFFFFULL) return set_error(WEDGE_ERANGE, "wedge_sample_close: too many tiles");
  if (A.alloc) {
    k_sample_close<1, true><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T);
    WEDGE_LAUNCH_CHECK("k_sample_close");
    return WEDGE_OK;
  }
  if (A.draw_only) {
    k_sample_close<1, false, true><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T);
    WEDGE_LAUNCH_CHECK("k_sample_close");
    return WEDGE_OK;
  }
  switch (U) {
    case 1: k_sample_close<1><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T); break;
    case 2: k_sample_close<2><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T); break;
    case 8: k_sample_close<8><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T); break;
    default: k_sample_close<4><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T); break;
  }
  WEDGE_LAUNCH_CHECK("k_sample_close");
  return WEDGE_OK;
}

int launch_persistent(const SamplerCtx& A, const uint64_t* task_k, const uint64_t* tile_begin,
                      uint64_t nrows, unsigned long long* ticket, const SampleTuning& t,
                      hipStream_t st) {
  int rc = fill<unsigned long long>(ticket, 1, 0ULL, st);
  if (rc) return rc;
  const unsigned grid = t.workgroups;
  switch (t.U) {
    case 1: k_sample_persistent<1><<<grid, kSampWG, 0, st>>>(A, task_k, tile_begin, nrows, ticket); break;
    case 2: k_sample_persistent<2><<<grid, kSampWG, 0, st>>>(A, task_k, tile_begin, nrows, ticket); break;
    case 8: k_sample_persistent<8><<<grid, kSampWG, 0, st>>>(A, task_k, tile_begin, nrows, ticket); break;
    default: k_sample_persistent<4><<<grid, kSampWG, 0, st>>>(A, task_k, tile_begin, nrows, ticket); break;
  }
  WEDGE_LAUNCH_CHECK("k_sample_persistent");
  return WEDGE_OK;
}

int sample_close_impl(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                      const void* d_index, uint32_t max_bins, const uint64_t* h_k,
                      uint64_t k_global, uint64_t seed, uint32_t graph_id, uint64_t* d_q,
                      uint64_t* d_probe_loads, wedge_sample_rec* d_dump, uint64_t dump_per_bin,
                      const SampleTuning* tuning, hipStream_t st,
                      const uint64_t* d_hash = nullptr, int hash_bits = 0,
                      bool draw_only = false) {
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_sample_close: n must be >= 1");
  if (max_bins == 0 || max_bins > 4096)
    return set_error(WEDGE_ERANGE, "wedge_sample_close: max_bins must be in [1, 4096]");
  if (!d_rowptr || !d_index || !d_q || !h_k)
    return set_error(WEDGE_EINVAL, "wedge_sample_close: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_index, 256) || !aligned(d_q, 8) ||
      !aligned(d_col, 4) || !aligned(d_probe_loads, 8) || !aligned(d_dump, 16))
    return set_error(WEDGE_EINVAL, "wedge_sample_close: misaligned pointer");
  uint64_t total = k_global;
  for (uint32_t b = 0; b < max_bins; ++b) {
    if (h_k[b] > (1ULL << 48))
      return set_error(WEDGE_ERANGE, "wedge_sample_close: k[%u] above 2^48", b);
    total += h_k[b];
  }
  if (k_global > (1ULL << 48))
    return set_error(WEDGE_ERANGE, "wedge_sample_close: k_global above 2^48");
  if (total > 0 && (m == 0 || (!d_col && !draw_only)))
    return set_error(WEDGE_EINVAL, "wedge_sample_close: samples requested of a graph without edges");
  if (d_dump && dump_per_bin == 0) d_dump = nullptr;
  if (draw_only && !d_dump) return set_error(WEDGE_EINVAL, "sample_draws: no record buffer");
  int rc;
  if ((rc = fill<uint64_t>(d_q, ((uint64_t)max_bins + 1) * 4, 0, st))) return rc;
  if (d_probe_loads && (rc = fill<uint64_t>(d_probe_loads, 1, 0, st))) return rc;
  SampleTuning t = tuning ? *tuning : default_tuning(total);
  normalise(t);
  SamplerCtx A;
  A.rowptr = d_rowptr;
  A.col = d_col;
  A.ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  A.seed = seed;
  A.spt = t.spt;
  A.dump_per_bin = dump_per_bin;
  A.q = d_q;
  A.probe_loads = d_probe_loads;
  A.dump = d_dump;
  A.class_cap = class_capacity(n, m, 1);
  A.n = n;
  A.max_bins = max_bins;
  A.num_graphs = 1;
  A.domain = kDomainSample;
  A.s_begin = 0;
  A.feat = nullptr;
  A.feat_stride = 0;
  A.omega = 2;
  A.tau = 1;
  A.closure = 1;
  A.hash = d_hash;
  A.hash_bits = hash_bits;
  A.draw_only = draw_only ? 1 : 0;
  TaskTable T;
  T.graph_word = graph_id;
  T.ntask = 0;
  for (uint32_t b = 0; b <= max_bins; ++b) {
    const bool glob = (b == max_bins);
    const uint64_t k = glob ? k_global : h_k[b];
    if (k == 0) continue;
    Task& K = T.task[T.ntask++];
    K.row = b;
    K.bword = glob ? kGlobalWord : b;
    K.k = k;
    K.s_begin = 0;
    K.slot = b;
    if (T.ntask == kMaxTasks) {
      if ((rc = launch_tasks(A, T, t.U, st))) return rc;
      T.ntask = 0;
    }
  }
  if (T.ntask > 0 && (rc = launch_tasks(A, T, t.U, st))) return rc;
  return WEDGE_OK;
}

int sample_draws(const uint64_t* d_rowptr, uint32_t n, uint64_t m, const void* d_index,
                 uint32_t max_bins, const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                 wedge_sample_rec* d_rec, uint64_t stride, uint64_t* d_q, hipStream_t st) {
  uint64_t kmax = k_global;
  for (uint32_t b = 0; b < max_bins; ++b) kmax = h_k[b] > kmax ? h_k[b] : kmax;
  if (stride < kmax) return set_error(WEDGE_ERANGE, "sample_draws: stride below a row's k");
  const SampleTuning t{1, 0, 0};
  return sample_close_impl(d_rowptr, nullptr, n, m, d_index, max_bins, h_k, k_global, seed, 0,
                           d_q, nullptr, d_rec, stride, &t, st, nullptr, 0, true);
}

// ------------------------------------------------------- allocation form
// Alg. phase2a on the index: the rows' vertex ranges, the per-vertex counts
// by probabilistic rounding, and the rows' realised totals.
constexpr uint64_t kDomainAlloc = 7;

// floor((hi * 2^64 + lo) / p) and the remainder, for hi < p (restoring
// division, one quotient bit per step).
__device__ inline void divmod_128_64(uint64_t hi, uint64_t lo, uint64_t p, uint64_t* q,
                                     uint64_t* r) {
  uint64_t rem = hi, quo = 0;
  for (int b = 63; b >= 0; --b) {
    const uint64_t top = rem >> 63;
    rem = (rem << 1) | (lo >> 63);
    lo <<= 1;
    if (top || rem >= p) {
      rem -= p;
      quo |= 1ULL << b;
    }
  }
  *q = quo;
  *r = rem;
}

// Row table: vertex range of every row with samples (its classes are
// consecutive in the centre order) and the rows' offsets in the count array.
__global__ void k_alloc_rows(IndexView ix, const uint64_t* __restrict__ k, uint32_t max_bins,
                             AllocRow* __restrict__ rows) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t off = 0;
  for (uint32_t f = 0; f <= max_bins; ++f) {
    const BinMeta M = ix.bins[f];
    AllocRow r{off, 0, 0, k[f]};
    if (k[f] > 0 && M.p_b > 0 && M.cls_lo < M.cls_hi) {
      const uint32_t j = M.cls_hi - 1;
      const uint64_t dj = ix.cls_deg[j];
      const uint64_t prev = j > 0 ? ix.cls_cumw[j - 1] : 0;
      const uint64_t last = (ix.cls_cumw[j] - prev) / (dj * (dj - 1) / 2);
      r.pos_lo = ix.cls_start[M.cls_lo];
      r.count = ix.cls_start[j] + last - r.pos_lo;
    } else {
      r.k = 0;
    }
    rows[f] = r;
    off += r.count;
  }
}

// q_v = floor(q*) + [U(p) < (C(d,2) k) mod p], q* = C(d,2) k / p, for every
// vertex of row blockIdx.y; the draw is word 2 of blocks (v, row word, g, r).
__global__ void k_alloc_round(const uint64_t* __restrict__ rowptr, IndexView ix,
                              const AllocRow* __restrict__ rows, uint32_t max_bins, uint64_t seed,
                              uint64_t domain, uint64_t gword, uint64_t* __restrict__ qv) {
  const uint32_t f = blockIdx.y;
  const AllocRow R = rows[f];
  if (R.count == 0) return;
  const uint64_t p = ix.bins[f].p_b;
  const uint64_t bw = f == max_bins ? kGlobalWord : f;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R.count; i += stride) {
    const uint32_t v = ix.vlist[R.pos_lo + i];
    const uint64_t d = rowptr[v + 1] - rowptr[v];
    const uint64_t a = d * (d - 1) / 2;
    uint64_t fl, rem;
    divmod_128_64(__umul64hi(a, R.k), a * R.k, p, &fl, &rem);
    const U64x4 o = philox4x64_10(v, bw, gword, 0, seed, domain);
    const uint64_t w = below_from(o.w[2], p, seed, domain, v, bw, gword, 2);
    qv[R.off + i] = fl + (w < rem ? 1 : 0);
  }
}

__global__ void k_alloc_totals(const AllocRow* __restrict__ rows, uint32_t nrows,
                               const uint64_t* __restrict__ pre, uint64_t* __restrict__ tot) {
  for (uint32_t f = threadIdx.x; f < nrows; f += blockDim.x) {
    const AllocRow R = rows[f];
    tot[f] = R.count ? pre[R.off + R.count] - pre[R.off] : 0;
  }
}

static int launch_centre_tasks(const SamplerCtx& A, TaskTable& T, const CentreArgs& C,
                               hipStream_t st) {
  uint64_t tiles = 0;
  for (uint32_t i = 0; i < T.ntask; ++i) {
    T.task[i].tile_begin = tiles;
    tiles += ceil_div(T.task[i].k, A.spt);
  }
  if (tiles == 0) return WEDGE_OK;
  if (tiles > 0x7FFFFFFFULL) return set_error(WEDGE_ERANGE, "centre means: too many tiles");
  k_centre_means<0><<<(unsigned)tiles, kSampWG, 0, st>>>(A, T, C);
  WEDGE_LAUNCH_CHECK("k_centre_means");
  return WEDGE_OK;
}

// Launch shapes picked by wedge_sample_close_autotune, per (device, n, m,
// max_bins): wedge_sample_close uses the pick for a graph of that size on
// that device from then on.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, uint32_t, uint64_t, uint32_t>, SampleTuning> g_tune;

static bool cached_tuning(uint32_t n, uint64_t m, uint32_t max_bins, SampleTuning* t) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(std::make_tuple(dev, n, m, max_bins));
  if (it == g_tune.end()) return false;
  *t = it->second;
  return true;
}

static SampleTuning tuning_of(const wedge_launch_shape& s) {
  SampleTuning t{s.lanes_in_flight, s.samples_per_tile, s.workgroups};
  normalise(t);
  return t;
}

}  // namespace wedge

using namespace wedge;

extern "C" int wedge_sample_close_autotune(const uint64_t* d_rowptr, const uint32_t* d_col,
                                           uint32_t n, uint64_t m, const void* d_index,
                                           uint32_t max_bins, const uint64_t* h_k,
                                           uint64_t k_global, uint64_t seed,
                                           const wedge_launch_shape* cands, int ncand, int reps,
                                           uint64_t* d_q_ref, uint64_t* d_q_try, float* h_ms,
                                           int* h_best, void* stream) {
  clear_error();
  if (!cands || ncand <= 0 || reps <= 0 || !d_q_ref || !d_q_try || !h_ms || !h_best)
    return set_error(WEDGE_EINVAL, "wedge_sample_close_autotune: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const size_t nq = ((size_t)max_bins + 1) * 4;
  std::vector<uint64_t> ref(nq), got(nq);
  hipEvent_t e0, e1;
  WEDGE_HIP_TRY(hipEventCreate(&e0));
  WEDGE_HIP_TRY(hipEventCreate(&e1));
  int rc = WEDGE_OK, best = -1;
  for (int c = 0; c < ncand && rc == WEDGE_OK; ++c) {
    const SampleTuning t = tuning_of(cands[c]);
    std::vector<float> ms(reps);
    uint64_t* q = c == 0 ? d_q_ref : d_q_try;
    for (int r = 0; r < reps && rc == WEDGE_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) { rc = set_error(WEDGE_EHIP, "event record"); break; }
      rc = sample_close_impl(d_rowptr, d_col, n, m, d_index, max_bins, h_k, k_global, seed, 0, q,
                             nullptr, nullptr, 0, &t, st);
      if (rc) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms[r], e0, e1) != hipSuccess) {
        rc = set_error(WEDGE_EHIP, "wedge_sample_close_autotune: event timing failed");
        break;
      }
    }
    if (rc) break;
    std::sort(ms.begin(), ms.end());
    h_ms[c] = ms[reps / 2];
    // every candidate must give the same counts (the result does not depend
    // on the launch shape)
    if (hipMemcpyAsync(c == 0 ? ref.data() : got.data(), q, nq * sizeof(uint64_t),
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = set_error(WEDGE_EHIP, "wedge_sample_close_autotune: copy of the counts failed");
      break;
    }
    if (c > 0 && got != ref) {
      rc = set_error(WEDGE_EINVAL, "wedge_sample_close_autotune: counts of candidate %d differ", c);
      break;
    }
    if (best < 0 || h_ms[c] < h_ms[best]) best = c;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  *h_best = best;
  int dev = 0;
  WEDGE_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[std::make_tuple(dev, n, m, max_bins)] = tuning_of(cands[best]);
  return WEDGE_OK;
}

extern "C" int wedge_sample_close_shape(uint32_t n, uint64_t m, uint32_t max_bins,
                                        wedge_launch_shape* h_shape) {
  clear_error();
  if (!h_shape) return set_error(WEDGE_EINVAL, "wedge_sample_close_shape: null pointer");
  SampleTuning t;
  if (!cached_tuning(n, m, max_bins, &t)) {
    t = default_tuning(0);
    normalise(t);
  }
  h_shape->lanes_in_flight = t.U;
  h_shape->samples_per_tile = (uint32_t)t.spt;
  h_shape->workgroups = t.workgroups;
  return WEDGE_OK;
}

extern "C" int wedge_sample_close(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                  uint64_t m, const void* d_index, uint32_t max_bins,
                                  const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                                  uint32_t graph_id, uint64_t* d_q, uint64_t* d_probe_loads,
                                  wedge_sample_rec* d_dump, uint64_t dump_per_bin, void* stream) {
  clear_error();
  if (validate_requested() && d_rowptr && d_q && n > 0 && (m == 0 || d_col)) {
    const int rc = validate_or_fail("wedge_sample_close", d_rowptr, d_col, n, m, d_q,
                                    (hipStream_t)stream);
    if (rc) return rc;
  }
  SampleTuning t;
  const bool tuned = cached_tuning(n, m, max_bins, &t);
  return sample_close_impl(d_rowptr, d_col, n, m, d_index, max_bins, h_k, k_global, seed,
                           graph_id, d_q, d_probe_loads, d_dump, dump_per_bin,
                           tuned ? &t : nullptr, (hipStream_t)stream);
}

extern "C" int wedge_sample_close_tuned(const uint64_t* d_rowptr, const uint32_t* d_col,
                                        uint32_t n, uint64_t m, const void* d_index,
                                        uint32_t max_bins, const uint64_t* h_k, uint64_t k_global,
                                        uint64_t seed, uint32_t graph_id, uint64_t* d_q,
                                        uint64_t* d_probe_loads, wedge_sample_rec* d_dump,
                                        uint64_t dump_per_bin, int lanes_in_flight,
                                        uint64_t samples_per_tile, void* stream) {
  clear_error();
  SampleTuning t{lanes_in_flight, samples_per_tile, 0};
  return sample_close_impl(d_rowptr, d_col, n, m, d_index, max_bins, h_k, k_global, seed,
                           graph_id, d_q, d_probe_loads, d_dump, dump_per_bin, &t,
                           (hipStream_t)stream);
}

extern "C" int wedge_sample_close_hashed(const uint64_t* d_rowptr, const uint32_t* d_col,
                                         uint32_t n, uint64_t m, const void* d_index,
                                         uint32_t max_bins, const uint64_t* h_k,
                                         uint64_t k_global, uint64_t seed, uint32_t graph_id,
                                         uint64_t* d_q, uint64_t* d_probe_loads,
                                         wedge_sample_rec* d_dump, uint64_t dump_per_bin,
                                         const uint64_t* d_table, uint32_t bits, void* stream) {
  clear_error();
  if (!d_table || !aligned(d_table, 8))
    return set_error(WEDGE_EINVAL, "wedge_sample_close_hashed: null or misaligned table");
  if (bits < 4 || bits > 40 || (1ULL << bits) < 2 * m)
    return set_error(WEDGE_ERANGE, "wedge_sample_close_hashed: 2^bits must be >= 2m");
  SampleTuning t;
  const bool tuned = cached_tuning(n, m, max_bins, &t);
  return sample_close_impl(d_rowptr, d_col, n, m, d_index, max_bins, h_k, k_global, seed,
                           graph_id, d_q, d_probe_loads, d_dump, dump_per_bin,
                           tuned ? &t : nullptr, (hipStream_t)stream, d_table, (int)bits);
}

extern "C" int wedge_sample_features(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                     uint64_t m, const void* d_index, uint32_t max_bins,
                                     uint32_t tau, uint64_t omega, const uint64_t* h_k,
                                     const uint64_t* h_s_begin, uint64_t seed, uint32_t domain,
                                     uint32_t graph_id, int closure, wedge_feature_rec* d_out,
                                     uint64_t out_stride, uint64_t* d_q, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_sample_features: n must be >= 1");
  if (max_bins == 0 || max_bins > 4096)
    return set_error(WEDGE_ERANGE, "wedge_sample_features: max_bins must be in [1, 4096]");
  if (tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_sample_features: need tau >= 1 and omega >= 2");
  if (!d_rowptr || !d_index || !h_k || !d_out)
    return set_error(WEDGE_EINVAL, "wedge_sample_features: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_index, 256) || !aligned(d_out, 16) ||
      !aligned(d_col, 4) || !aligned(d_q, 8))
    return set_error(WEDGE_EINVAL, "wedge_sample_features: misaligned pointer");
  uint64_t total = 0;
  for (uint32_t r = 0; r <= max_bins; ++r) {
    if (h_k[r] > out_stride)
      return set_error(WEDGE_ERANGE, "wedge_sample_features: k[%u] > out_stride", r);
    if (h_s_begin && h_s_begin[r] + h_k[r] > (1ULL << 48))
      return set_error(WEDGE_ERANGE, "wedge_sample_features: s_begin[%u] + k beyond 2^48", r);
    total += h_k[r];
  }
  if (total > 0 && (m == 0 || !d_col))
    return set_error(WEDGE_EINVAL, "wedge_sample_features: samples of a graph without edges");
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (d_q && (rc = fill<uint64_t>(d_q, ((uint64_t)max_bins + 1) * 4, 0, st))) return rc;
  uint64_t* q = d_q;
  SampleTuning t = default_tuning(total);
  normalise(t);
  SamplerCtx A;
  A.rowptr = d_rowptr;
  A.col = d_col;
  A.ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  A.seed = seed;
  A.spt = t.spt;
  A.dump_per_bin = 0;
  A.q = q;
  A.probe_loads = nullptr;
  A.dump = nullptr;
  A.class_cap = class_capacity(n, m, 1);
  A.n = n;
  A.max_bins = max_bins;
  A.num_graphs = 1;
  A.domain = domain;
  A.s_begin = 0;
  A.feat = d_out;
  A.feat_stride = out_stride;
  A.omega = omega;
  A.tau = tau;
  A.closure = closure ? 1 : 0;
  TaskTable T;
  T.graph_word = graph_id;
  T.ntask = 0;
  uint64_t slot = 0;
  for (uint32_t b = 0; b <= max_bins; ++b) {
    if (h_k[b] == 0) continue;
    Task& K = T.task[T.ntask++];
    K.row = b;
    K.bword = (b == max_bins) ? kGlobalWord : b;
    K.k = h_k[b];
    K.s_begin = h_s_begin ? h_s_begin[b] : 0;
    K.slot = slot++;
    if (T.ntask == kMaxTasks) {
      if ((rc = launch_tasks(A, T, t.U, st))) return rc;
      T.ntask = 0;
    }
  }
  if (T.ntask > 0 && (rc = launch_tasks(A, T, t.U, st))) return rc;
  return WEDGE_OK;
}

struct AllocWorkspace {
  AllocRow* rows;
  uint64_t* k;
  uint64_t* tot;
  uint64_t* qv;
  uint64_t* scan_ws;
};

static size_t alloc_layout(uint32_t n, uint32_t max_bins, AllocWorkspace* w, void* base) {
  char* c = (char*)base;
  size_t off = 0;
  const uint64_t rows = (uint64_t)max_bins + 1;
  const uint64_t N = 2 * (uint64_t)n + 1;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;  // sizing calls pass no base
    off += round_up(bytes, 256);
    return p;
  };
  AllocWorkspace x;
  x.rows = (AllocRow*)take(rows * sizeof(AllocRow));
  x.k = (uint64_t*)take(rows * 8);
  x.tot = (uint64_t*)take(rows * 8);
  x.qv = (uint64_t*)take(N * 8);
  x.scan_ws = (uint64_t*)take(scan_ws_elems(N) * 8);
  if (w) *w = x;
  return off;
}

extern "C" size_t wedge_sample_alloc_workspace(uint32_t n, uint32_t max_bins) {
  return alloc_layout(n, max_bins, nullptr, nullptr);
}

extern "C" int wedge_sample_alloc(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                  uint64_t m, const void* d_index, uint32_t max_bins,
                                  const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                                  uint64_t* d_q, uint64_t* h_totals, wedge_sample_rec* d_dump,
                                  uint64_t dump_per_bin, void* d_workspace,
                                  size_t workspace_bytes, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_sample_alloc: n must be >= 1");
  if (max_bins == 0 || max_bins > 4096)
    return set_error(WEDGE_ERANGE, "wedge_sample_alloc: max_bins must be in [1, 4096]");
  if (!d_rowptr || !d_index || !h_k || !d_q || !h_totals || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_sample_alloc: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_index, 256) || !aligned(d_q, 8) ||
      !aligned(d_col, 4) || !aligned(d_dump, 16) || !aligned(d_workspace, 256))
    return set_error(WEDGE_EINVAL, "wedge_sample_alloc: misaligned pointer");
  if (workspace_bytes < wedge_sample_alloc_workspace(n, max_bins))
    return set_error(WEDGE_EWORKSPACE, "wedge_sample_alloc: workspace %zu < %zu bytes",
                     workspace_bytes, wedge_sample_alloc_workspace(n, max_bins));
  uint64_t total = k_global;
  for (uint32_t b = 0; b < max_bins; ++b) {
    if (h_k[b] > (1ULL << 48))
      return set_error(WEDGE_ERANGE, "wedge_sample_alloc: k[%u] above 2^48", b);
    total += h_k[b];
  }
  if (k_global > (1ULL << 48))
    return set_error(WEDGE_ERANGE, "wedge_sample_alloc: k_global above 2^48");
  if (total > 0 && (m == 0 || !d_col))
    return set_error(WEDGE_EINVAL, "wedge_sample_alloc: samples requested of a graph without edges");
  if (d_dump && dump_per_bin == 0) d_dump = nullptr;
  hipStream_t st = (hipStream_t)stream;
  AllocWorkspace w;
  alloc_layout(n, max_bins, &w, d_workspace);
  const uint32_t rows = max_bins + 1;
  std::vector<uint64_t> hk(rows);
  for (uint32_t b = 0; b < max_bins; ++b) hk[b] = h_k[b];
  hk[max_bins] = k_global;
  const IndexView ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  const uint64_t N = 2 * (uint64_t)n + 1;
  int rc;
  if ((rc = fill<uint64_t>(d_q, (uint64_t)rows * 4, 0, st))) return rc;
  if ((rc = fill<uint64_t>(w.qv, N, 0, st))) return rc;
  WEDGE_HIP_TRY(hipMemcpyAsync(w.k, hk.data(), rows * 8, hipMemcpyHostToDevice, st));
  k_alloc_rows<<<1, 64, 0, st>>>(ix, w.k, max_bins, w.rows);
  WEDGE_LAUNCH_CHECK("k_alloc_rows");
  k_alloc_round<<<dim3(256, rows), 256, 0, st>>>(d_rowptr, ix, w.rows, max_bins, seed,
                                                 kDomainAlloc, 0, w.qv);
  WEDGE_LAUNCH_CHECK("k_alloc_round");
  rc = scan_apply<uint64_t>(LoadArray<uint64_t>{w.qv}, StoreExclusive<uint64_t>{w.qv}, N,
                            w.scan_ws, st);
  if (rc) return rc;
  k_alloc_totals<<<1, 256, 0, st>>>(w.rows, rows, w.qv, w.tot);
  WEDGE_LAUNCH_CHECK("k_alloc_totals");
  WEDGE_HIP_TRY(hipMemcpyAsync(h_totals, w.tot, rows * 8, hipMemcpyDeviceToHost, st));
  WEDGE_HIP_TRY(hipStreamSynchronize(st));
  uint64_t drawn = 0;
  for (uint32_t f = 0; f < rows; ++f) drawn += h_totals[f];
  SampleTuning t = default_tuning(drawn);
  normalise(t);
  SamplerCtx A;
  A.rowptr = d_rowptr;
  A.col = d_col;
  A.ix = ix;
  A.seed = seed;
  A.spt = t.spt;
  A.dump_per_bin = dump_per_bin;
  A.q = d_q;
  A.probe_loads = nullptr;
  A.dump = d_dump;
  A.class_cap = class_capacity(n, m, 1);
  A.n = n;
  A.max_bins = max_bins;
  A.num_graphs = 1;
  A.domain = kDomainAlloc;
  A.s_begin = 0;
  A.feat = nullptr;
  A.feat_stride = 0;
  A.omega = 2;
  A.tau = 1;
  A.closure = 1;
  A.alloc = w.rows;
  A.alloc_pre = w.qv;
  TaskTable T;
  T.graph_word = 0;
  T.ntask = 0;
  for (uint32_t b = 0; b < rows; ++b) {
    if (h_totals[b] == 0) continue;
    Task& K = T.task[T.ntask++];
    K.row = b;
    K.bword = (b == max_bins) ? kGlobalWord : b;
    K.k = h_totals[b];
    K.s_begin = 0;
    K.slot = b;
    if (T.ntask == kMaxTasks) {
      if ((rc = launch_tasks(A, T, t.U, st))) return rc;
      T.ntask = 0;
    }
  }
  if (T.ntask > 0 && (rc = launch_tasks(A, T, t.U, st))) return rc;
  return WEDGE_OK;
}

extern "C" size_t wedge_cv_centre_means_workspace(uint64_t total_draws) {
  return 256 + round_up(total_draws * 24, 256);
}

extern "C" int wedge_cv_centre_means(const uint64_t* d_rowptr, const uint32_t* d_col,
                                     uint32_t n, uint64_t m, const void* d_index,
                                     uint32_t max_bins, uint32_t tau, uint64_t omega,
                                     const uint64_t* h_k, const uint64_t* h_s_begin,
                                     uint64_t seed, uint32_t domain, uint32_t graph_id,
                                     const void* d_census, const float* d_gtable, float* d_out,
                                     uint64_t out_stride, uint32_t* d_vout, void* d_workspace,
                                     size_t workspace_bytes, void* stream) {
  clear_error();
  if (n == 0) return set_error(WEDGE_ERANGE, "wedge_cv_centre_means: n must be >= 1");
  if (max_bins == 0 || max_bins > 4096 || tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_cv_centre_means: bad max_bins, tau or omega");
  if (!d_rowptr || !d_index || !h_k || !d_census || !d_gtable || !d_out || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_cv_centre_means: null pointer");
  if (!aligned(d_rowptr, 8) || !aligned(d_index, 256) || !aligned(d_census, 256) ||
      !aligned(d_workspace, 256) || !aligned(d_out, 4))
    return set_error(WEDGE_EINVAL, "wedge_cv_centre_means: misaligned pointer");
  uint64_t total = 0;
  for (uint32_t r = 0; r <= max_bins; ++r) {
    if (h_k[r] > out_stride)
      return set_error(WEDGE_ERANGE, "wedge_cv_centre_means: k[%u] > out_stride", r);
    if (h_s_begin && h_s_begin[r] + h_k[r] > (1ULL << 48))
      return set_error(WEDGE_ERANGE, "wedge_cv_centre_means: s_begin[%u] + k beyond 2^48", r);
    total += h_k[r];
  }
  if (total == 0) return WEDGE_OK;
  if (m == 0 || !d_col)
    return set_error(WEDGE_EINVAL, "wedge_cv_centre_means: draws of a graph without edges");
  if (workspace_bytes < wedge_cv_centre_means_workspace(total))
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_centre_means: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  CentreArgs C;
  C.key_of = census_key_of(d_census, max_bins);
  C.gtable = d_gtable;
  C.out = d_out;
  C.vout = d_vout;
  C.stride = out_stride;
  C.queued = (unsigned long long*)d_workspace;
  C.queue = (uint64_t*)((char*)d_workspace + 256);
  C.capacity = total;
  int rc = fill<unsigned long long>(C.queued, 1, 0, st);
  if (rc) return rc;
  SamplerCtx A;
  A.rowptr = d_rowptr;
  A.col = d_col;
  A.ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  A.seed = seed;
  A.spt = (uint64_t)kSampWG;
  A.dump_per_bin = 0;
  A.q = nullptr;
  A.probe_loads = nullptr;
  A.dump = nullptr;
  A.class_cap = class_capacity(n, m, 1);
  A.n = n;
  A.max_bins = max_bins;
  A.num_graphs = 1;
  A.domain = domain;
  A.s_begin = 0;
  A.feat = nullptr;
  A.feat_stride = 0;
  A.omega = omega;
  A.tau = tau;
  A.closure = 0;
  TaskTable T;
  T.graph_word = graph_id;
  T.ntask = 0;
  uint64_t slot = 0;
  for (uint32_t b = 0; b <= max_bins; ++b) {
    if (h_k[b] == 0) continue;
    Task& K = T.task[T.ntask++];
    K.row = b;
    K.bword = (b == max_bins) ? kGlobalWord : b;
    K.k = h_k[b];
    K.s_begin = h_s_begin ? h_s_begin[b] : 0;
    K.slot = slot++;
    if (T.ntask == kMaxTasks) {
      if ((rc = launch_centre_tasks(A, T, C, st))) return rc;
      T.ntask = 0;
    }
  }
  if (T.ntask > 0 && (rc = launch_centre_tasks(A, T, C, st))) return rc;
  k_centre_wide<<<1024, 256, 0, st>>>(A, C);
  WEDGE_LAUNCH_CHECK("k_centre_wide");
  return WEDGE_OK;
}
