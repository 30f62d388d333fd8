// Exact mean of the control-variate network over all wedges of every bin.
//
// The network reads (bin, K(d_v), K(min(d_a,d_c)), K(max(d_a,d_c))) with
// K(d) = floor(8 L(d)) the log-degree bucket, so its mean over the wedges
// of bin b is a finite sum: mu_b = (1/p_b) sum over keys (b, K(d_v)) and
// bucket pairs (i <= j) of census(b, K(d_v), i, j) * g(b, K(d_v), i, j).
// The census counts, for each key, the wedges whose endpoints fall in
// buckets (i, j).  For a centre v with neighbour-bucket histogram h_v it
// adds h_v[i] h_v[j] to (i, j) and C(h_v[i], 2) to (i, i): summed over the
// centres of a key that is the Gram matrix of their histograms.
//
// Work layout.  A byte array holds every vertex's bucket, so a neighbour
// costs one byte gather (the array is small enough to stay in the caches).
// Workgroups take equal shares of the total degree 2m along the centre order
// (vertices by degree; the split is found on the per-degree class table), and
// walk their share one key segment at a time.  A segment's largest degree
// picks the mode: one lane per centre for small degrees (every neighbour
// pair adds one wedge), one wave per centre for medium degrees (bucket
// histogram in LDS, then every pair of non-empty buckets), the whole
// workgroup per centre for hubs.  Pair counts with both buckets below 160
// (degrees below 2^20) accumulate in a 64-bit LDS table of the segment,
// flushed with one global atomic per non-zero entry; rarer pairs go to the
// global table directly.
#include "common.hpp"
#include "scan.hpp"

namespace wedge {

constexpr uint32_t kBuckets = 256;
constexpr uint32_t kPairs = kBuckets * (kBuckets + 1) / 2;     // 32896
constexpr uint32_t kLdsBuckets = 160;  // degrees below 2^20
constexpr uint32_t kLdsPairs = kLdsBuckets * (kLdsBuckets + 1) / 2;  // 12880
constexpr uint32_t kCensusWG = 512;
constexpr uint32_t kCensusWaves = kCensusWG / 64;
constexpr uint32_t kLaneMaxDeg = 64;    // a lane per centre up to this degree
constexpr uint32_t kWaveMaxDeg = 2048;  // a wave per centre up to this degree
constexpr uint32_t kNoKey = 0xFFFFFFFFu;

__device__ __host__ inline uint32_t bucket_of(uint64_t d) {
  if (d == 0) return 0;
  const uint32_t e = 63 - (uint32_t)__builtin_clzll(d);
  const uint64_t p = 1ULL << e;
  return 8 * e + (uint32_t)(((d - p) * 8) >> e);
}

// smallest degree of bucket k (k in [0, 256]); 2^32 for k = 256
__device__ __host__ inline uint64_t bucket_rep(uint32_t k) {
  if (k >= kBuckets) return 1ULL << 32;
  const uint32_t e = k >> 3, f = k & 7;
  const uint64_t p = 1ULL << e;
  return p + ((uint64_t)f * p + 7) / 8;
}

__device__ inline uint32_t pair_index(uint32_t i, uint32_t j) { return j * (j + 1) / 2 + i; }

struct CensusView {
  uint32_t* nkeys;       // [1]
  uint32_t* key_of;      // [max_bins * 256]: key id of (bin, bucket) or kNoKey
  uint32_t* key_bin;     // [cap]
  uint32_t* key_bucket;  // [cap]
  uint32_t* key_rep;     // [cap] a degree in both the bin and the bucket
  uint64_t* table;       // [cap][kPairs]
  uint8_t* vbucket;      // [n] bucket of every vertex's degree
  uint64_t* cls_work;    // [class_cap + 1] total degree of the classes before j
  uint32_t cap;
};

inline uint32_t census_cap(uint32_t max_bins) { return kBuckets + max_bins + 1; }

// The key list and the table come first, so their offsets depend only on
// max_bins; the per-graph scratch follows.
static size_t census_layout(uint32_t max_bins, uint64_t n, uint64_t class_cap, CensusView* v,
                            void* base) {
  const uint32_t cap = census_cap(max_bins);
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;  // sizing calls pass no base
    off += round_up(bytes, 256);
    return (void*)p;
  };
  void* nk = take(8);
  void* ko = take((size_t)max_bins * kBuckets * 4);
  void* kb = take((size_t)cap * 4);
  void* kk = take((size_t)cap * 4);
  void* kr = take((size_t)cap * 4);
  void* tb = take((size_t)cap * kPairs * 8);
  void* vb = take(n ? n : 1);
  void* cw = take((class_cap + 1) * 8);
  if (v) {
    v->nkeys = (uint32_t*)nk;
    v->key_of = (uint32_t*)ko;
    v->key_bin = (uint32_t*)kb;
    v->key_bucket = (uint32_t*)kk;
    v->key_rep = (uint32_t*)kr;
    v->table = (uint64_t*)tb;
    v->vbucket = (uint8_t*)vb;
    v->cls_work = (uint64_t*)cw;
    v->cap = cap;
  }
  return off;
}

// The (bin, bucket) keys that degrees >= 2 can take, numbered in increasing
// degree order (bucket, then bin: both are monotone in the degree).  Thread k
// takes bucket k; an exclusive scan of the per-bucket key counts numbers them.
__global__ __launch_bounds__(256) void k_census_keys(CensusView C, uint32_t tau, uint64_t omega,
                                                     uint32_t max_bins) {
  __shared__ uint32_t s_w[4];
  const uint32_t k = threadIdx.x, lane = k & 63, wave = k >> 6;
  for (uint32_t i = k; i < max_bins * kBuckets; i += blockDim.x) C.key_of[i] = kNoKey;
  uint64_t lo = bucket_rep(k), hi = bucket_rep(k + 1) - 1;
  if (lo < 2) lo = 2;
  if (hi > 0xFFFFFFFFULL) hi = 0xFFFFFFFFULL;
  uint32_t b0 = 0, cnt = 0;
  if (hi >= 2 && lo <= hi) {
    b0 = bin_id_capped(lo, tau, omega, max_bins);
    const uint32_t b1 = bin_id_capped(hi, tau, omega, max_bins);  // bins b0 .. b1 hold degrees here
    if (b0 < max_bins) cnt = (b1 < max_bins ? b1 : max_bins - 1) - b0 + 1;
  }
  const uint32_t incl = wave_incl_scan(cnt, (int)lane);
  if (lane == 63) s_w[wave] = incl;
  __syncthreads();
  uint32_t first = incl - cnt;
  for (uint32_t w = 0; w < wave; ++w) first += s_w[w];
  const uint32_t total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
  for (uint32_t j = 0; j < cnt; ++j) {
    const uint32_t id = first + j;
    if (id >= C.cap) break;
    const uint32_t b = b0 + j;
    const uint64_t blo = bin_lo_deg(b, tau, omega);
    C.key_of[b * kBuckets + k] = id;
    C.key_bin[id] = b;
    C.key_bucket[id] = k;
    C.key_rep[id] = (uint32_t)(blo > lo ? blo : lo);
  }
  if (k == 0) *C.nkeys = total < C.cap ? total : C.cap;
}

__global__ void k_vertex_bucket(const uint64_t* __restrict__ rowptr, uint64_t n,
                                uint8_t* __restrict__ vb) {
  uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; v < n; v += stride) vb[v] = (uint8_t)bucket_of(rowptr[v + 1] - rowptr[v]);
}

// cls_work[j] = sum over classes c < j of count_c * deg_c (exclusive), for
// j = 0 .. num_classes; one workgroup.
__global__ __launch_bounds__(1024) void k_class_work(IndexView ix, uint64_t n,
                                                     uint64_t* __restrict__ cls_work) {
  __shared__ uint64_t s_w[16];
  const uint32_t nc = ix.hdr->num_classes;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t run = 0;
  for (uint32_t base = 0; base < nc; base += 1024) {
    const uint32_t j = base + tid;
    uint64_t w = 0;
    if (j < nc) {
      const uint64_t end = (j + 1 < nc) ? ix.cls_start[j + 1] : n;
      w = (end - ix.cls_start[j]) * (uint64_t)ix.cls_deg[j];
    }
    const uint64_t incl = wave_incl_scan(w, lane);
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int q = 0; q < 16; ++q) {
      if (q < wave) before += s_w[q];
      tot += s_w[q];
    }
    if (j < nc) cls_work[j] = run + before + incl - w;
    run += tot;
    __syncthreads();
  }
  if (tid == 0) cls_work[nc] = run;
}

// Smallest centre-order position whose preceding degrees sum to >= w.
__device__ inline uint64_t position_of_work(const IndexView& ix, const uint64_t* cls_work,
                                            uint32_t nc, uint64_t n, uint64_t w) {
  if (w == 0) return 0;
  if (w > cls_work[nc]) return n;
  uint32_t lo = 0, hi = nc;  // last j with cls_work[j] < w
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (cls_work[mid] < w) lo = mid; else hi = mid;
  }
  const uint64_t d = ix.cls_deg[lo];
  const uint64_t end = (lo + 1 < nc) ? ix.cls_start[lo + 1] : n;
  uint64_t p = ix.cls_start[lo] + (d ? (w - cls_work[lo] + d - 1) / d : 0);
  return p < end ? p : end;
}

// key of a centre of degree d, or kNoKey (d < 2, or a bin beyond the table)
__device__ inline uint32_t key_of_degree(const CensusView& C, uint64_t d, uint32_t tau,
                                         uint64_t omega, uint32_t max_bins) {
  if (d < 2) return kNoKey;
  const uint32_t b = bin_id_capped(d, tau, omega, max_bins);
  if (b >= max_bins) return kNoKey;
  return C.key_of[b * kBuckets + bucket_of(d)];
}

__device__ inline void add_pair(unsigned long long* s_tab, uint64_t* gtab, uint32_t bi,
                                uint32_t bj, uint64_t cnt) {
  if (bi > bj) {
    const uint32_t t = bi;
    bi = bj;
    bj = t;
  }
  if (bj < kLdsBuckets)
    atomicAdd(&s_tab[pair_index(bi, bj)], (unsigned long long)cnt);
  else
    atomicAdd((unsigned long long*)&gtab[pair_index(bi, bj)], (unsigned long long)cnt);
}

// (i, j) of the t-th pair i <= j of a list, t < u (u + 1) / 2
__device__ inline void pair_of(uint32_t t, uint32_t* i, uint32_t* j) {
  uint32_t jj = (uint32_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (jj * (jj + 1) / 2 > t) --jj;
  while ((jj + 1) * (jj + 2) / 2 <= t) ++jj;
  *j = jj;
  *i = t - jj * (jj + 1) / 2;
}

__global__ __launch_bounds__(kCensusWG) void k_census(const uint64_t* __restrict__ rowptr,
                                                      const uint32_t* __restrict__ col,
                                                      IndexView ix, uint64_t n, uint64_t work,
                                                      uint32_t nchunks, uint32_t tau,
                                                      uint64_t omega, uint32_t max_bins,
                                                      CensusView C) {
  __shared__ unsigned long long s_tab[kLdsPairs];              // 103040 B
  __shared__ uint32_t s_hist[kCensusWaves][kBuckets];           // 8 KB
  __shared__ uint16_t s_list[kCensusWaves][kBuckets];           // 4 KB
  __shared__ uint32_t s_cnt[kCensusWaves][kBuckets];            // 8 KB
  __shared__ uint8_t s_lane[kLaneMaxDeg][kCensusWG];            // 32 KB
  __shared__ uint64_t s_seg[3];
  __shared__ uint32_t s_wsum[kCensusWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t nc = ix.hdr->num_classes;
  const uint64_t p0 = position_of_work(ix, C.cls_work, nc, n, (uint64_t)blockIdx.x * work);
  const uint64_t p1 = (blockIdx.x + 1 == nchunks)
                          ? n
                          : position_of_work(ix, C.cls_work, nc, n,
                                             (uint64_t)(blockIdx.x + 1) * work);
  if (p0 >= p1) return;
  for (uint32_t i = tid; i < kLdsPairs; i += kCensusWG) s_tab[i] = 0;
  for (uint32_t i = tid; i < kCensusWaves * kBuckets; i += kCensusWG) (&s_hist[0][0])[i] = 0;
  __syncthreads();
  const uint32_t nkeys = *C.nkeys;
  uint64_t seg = p0;
  while (seg < p1) {
    if (wave == 0) {
      // class holding seg, then the first later class with another key
      uint32_t lo = 0, hi = nc;
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ix.cls_start[mid] <= seg) lo = mid; else hi = mid;
      }
      const uint32_t key0 = key_of_degree(C, ix.cls_deg[lo], tau, omega, max_bins);
      uint64_t end = n;
      uint32_t last = lo;
      for (uint32_t c = lo + 1; c < nc; c += 64) {
        const uint32_t cj = c + lane;
        const bool other =
            cj < nc && key_of_degree(C, ix.cls_deg[cj], tau, omega, max_bins) != key0;
        const uint64_t ball = __ballot(other);
        if (ball) {
          const uint32_t first = c + (uint32_t)__builtin_ctzll(ball);
          end = ix.cls_start[first];
          last = first - 1;
          break;
        }
        last = (c + 64 < nc) ? c + 63 : nc - 1;
      }
      if (lane == 0) {
        s_seg[0] = end < p1 ? end : p1;
        s_seg[1] = key0;
        s_seg[2] = ix.cls_deg[last];
      }
    }
    __syncthreads();
    const uint64_t seg_end = s_seg[0];
    const uint32_t key = (uint32_t)s_seg[1];
    const uint64_t dmax = s_seg[2];
    __syncthreads();
    if (key == kNoKey || key >= nkeys) {  // centres without wedges (or beyond the bins)
      seg = seg_end;
      continue;
    }
    uint64_t* gtab = C.table + (uint64_t)key * kPairs;
    if (dmax <= kLaneMaxDeg) {
      // a lane per centre: every pair of its neighbours is one wedge
      for (uint64_t pos = seg + tid; pos < seg_end; pos += kCensusWG) {
        const uint64_t r0 = ix.vrow[pos];
        const uint32_t v = ix.vlist[pos];
        const uint32_t d = (uint32_t)(rowptr[v + 1] - r0);
        // neighbour buckets, eight independent gathers at a time
        for (uint32_t x0 = 0; x0 < d; x0 += 8) {
          uint32_t nb[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) nb[q] = x0 + q < d ? col[r0 + x0 + q] : 0;
          uint8_t bk[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) bk[q] = x0 + q < d ? C.vbucket[nb[q]] : 0;
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (x0 + q < d) s_lane[x0 + q][tid] = bk[q];
        }
        for (uint32_t x = 1; x < d; ++x) {
          const uint32_t bx = s_lane[x][tid];
          for (uint32_t y = 0; y < x; ++y) add_pair(s_tab, gtab, s_lane[y][tid], bx, 1);
        }
      }
    } else if (dmax <= kWaveMaxDeg) {
      // a wave per centre
      for (uint64_t pos = seg + wave; pos < seg_end; pos += kCensusWaves) {
        const uint64_t r0 = ix.vrow[pos];
        const uint32_t v = ix.vlist[pos];
        const uint64_t r1 = rowptr[v + 1];
        // four independent gathers per lane at a time
        for (uint64_t x0 = r0 + lane; x0 < r1; x0 += 4 * 64) {
          uint32_t nb[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) nb[q] = x0 + 64 * q < r1 ? col[x0 + 64 * q] : 0;
          uint32_t bk[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) bk[q] = x0 + 64 * q < r1 ? C.vbucket[nb[q]] : 0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (x0 + 64 * q < r1) atomicAdd(&s_hist[wave][bk[q]], 1u);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        // compact the non-empty buckets in increasing order
        uint32_t h[4];
        uint32_t nz = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          h[t] = s_hist[wave][lane * 4 + t];
          nz += h[t] > 0;
        }
        const uint32_t pre = wave_incl_scan(nz, lane);
        const uint32_t u = __shfl(pre, 63, 64);
        uint32_t at = pre - nz;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (h[t] > 0) {
            s_list[wave][at] = (uint16_t)(lane * 4 + t);
            s_cnt[wave][at] = h[t];
            ++at;
          }
          s_hist[wave][lane * 4 + t] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_s_waitcnt(0);
        const uint32_t np = u * (u + 1) / 2;
        for (uint32_t t = lane; t < np; t += 64) {
          uint32_t i, j;
          pair_of(t, &i, &j);
          const uint64_t hi_ = s_cnt[wave][i], hj = s_cnt[wave][j];
          const uint64_t cnt = (i == j) ? hi_ * (hi_ - 1) / 2 : hi_ * hj;
          if (cnt) add_pair(s_tab, gtab, s_list[wave][i], s_list[wave][j], cnt);
        }
        __builtin_amdgcn_wave_barrier();
      }
    } else {
      // the whole workgroup per centre (hubs): each wave fills its own
      // histogram row and the rows are summed
      for (uint64_t pos = seg; pos < seg_end; ++pos) {
        const uint64_t r0 = ix.vrow[pos];
        const uint32_t v = ix.vlist[pos];
        const uint64_t r1 = rowptr[v + 1];
        for (uint64_t x0 = r0 + tid; x0 < r1; x0 += 4 * kCensusWG) {
          uint32_t nb[4];
#pragma unroll
          for (int q = 0; q < 4; ++q)
            nb[q] = x0 + kCensusWG * q < r1 ? col[x0 + kCensusWG * q] : 0;
          uint32_t bk[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) bk[q] = x0 + kCensusWG * q < r1 ? C.vbucket[nb[q]] : 0;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (x0 + kCensusWG * q < r1) atomicAdd(&s_hist[wave][bk[q]], 1u);
        }
        __syncthreads();
        uint32_t h = 0, nz = 0;
        if (tid < (int)kBuckets) {
          for (int w = 0; w < (int)kCensusWaves; ++w) h += s_hist[w][tid];
          nz = h > 0;
        }
        const uint32_t pre = wave_incl_scan(nz, lane);
        if (lane == 63) s_wsum[wave] = pre;
        __syncthreads();
        uint32_t before = 0, u = 0;
        for (int q = 0; q < (int)(kBuckets / 64); ++q) {
          if (q < wave) before += s_wsum[q];
          u += s_wsum[q];
        }
        if (tid < (int)kBuckets) {
          if (h > 0) {
            s_list[1][before + pre - 1] = (uint16_t)tid;
            s_cnt[1][before + pre - 1] = h;
          }
          for (int w = 0; w < (int)kCensusWaves; ++w) s_hist[w][tid] = 0;
        }
        __syncthreads();
        const uint32_t np = u * (u + 1) / 2;
        for (uint32_t t = tid; t < np; t += kCensusWG) {
          uint32_t i, j;
          pair_of(t, &i, &j);
          const uint64_t hi_ = s_cnt[1][i], hj = s_cnt[1][j];
          const uint64_t cnt = (i == j) ? hi_ * (hi_ - 1) / 2 : hi_ * hj;
          if (cnt) add_pair(s_tab, gtab, s_list[1][i], s_list[1][j], cnt);
        }
        __syncthreads();
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < kLdsPairs; i += kCensusWG) {
      const unsigned long long x = s_tab[i];
      if (x) {
        atomicAdd((unsigned long long*)&gtab[i], x);
        s_tab[i] = 0;
      }
    }
    __syncthreads();
    seg = seg_end;
  }
}

// Records of every (key, bucket pair): representative degrees of the key's
// centre and of the two endpoint buckets, and the key's bin.
__global__ void k_census_records(CensusView C, wedge_feature_rec* __restrict__ rec) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nk = *C.nkeys;
  if (t >= (uint64_t)nk * kPairs) return;
  const uint32_t key = (uint32_t)(t / kPairs), p = (uint32_t)(t % kPairs);
  uint32_t j = (uint32_t)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > p) --j;
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  const uint32_t i = p - j * (j + 1) / 2;
  wedge_feature_rec r;
  r.dv = C.key_rep[key];
  const uint64_t ri = bucket_rep(i), rj = bucket_rep(j);
  r.dlo = (uint32_t)(ri > 0xFFFFFFFFULL ? 0xFFFFFFFFULL : ri);
  r.dhi = (uint32_t)(rj > 0xFFFFFFFFULL ? 0xFFFFFFFFULL : rj);
  r.bin = (uint16_t)C.key_bin[key];
  r.closed = 0;
  r.cls = 0;
  rec[t] = r;
}

// sum over a key's pairs of count * g in a fixed order (deterministic)
__global__ __launch_bounds__(256) void k_census_dot(CensusView C, const float* __restrict__ g,
                                                    double* __restrict__ key_sum,
                                                    uint64_t* __restrict__ key_count) {
  __shared__ double s_d[256];
  __shared__ unsigned long long s_c[256];
  const uint32_t key = blockIdx.x;
  if (key >= *C.nkeys) return;
  const uint64_t* T = C.table + (uint64_t)key * kPairs;
  const float* G = g + (uint64_t)key * kPairs;
  double acc = 0.0;
  unsigned long long cnt = 0;
  for (uint32_t p = threadIdx.x; p < kPairs; p += 256) {
    const uint64_t c = T[p];
    if (c) {
      acc += (double)c * (double)G[p];
      cnt += c;
    }
  }
  s_d[threadIdx.x] = acc;
  s_c[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s_d[threadIdx.x] += s_d[threadIdx.x + off];
      s_c[threadIdx.x] += s_c[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    key_sum[key] = s_d[0];
    key_count[key] = s_c[0];
  }
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_cv_census_bytes(uint32_t n, uint64_t m, uint32_t max_bins) {
  return census_layout(max_bins, n, class_capacity(n, m, 1), nullptr, nullptr);
}

extern "C" int wedge_cv_census(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                               uint64_t m, const void* d_index, uint32_t max_bins, uint32_t tau,
                               uint64_t omega, void* d_census, size_t census_bytes,
                               void* stream) {
  clear_error();
  if (n == 0 || max_bins == 0 || max_bins > 4096 || tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_cv_census: bad n, max_bins, tau or omega");
  if (!d_rowptr || !d_index || !d_census || (m > 0 && !d_col))
    return set_error(WEDGE_EINVAL, "wedge_cv_census: null pointer");
  if (!aligned(d_census, 256) || !aligned(d_index, 256) || !aligned(d_rowptr, 8))
    return set_error(WEDGE_EINVAL, "wedge_cv_census: misaligned pointer");
  if (census_bytes < wedge_cv_census_bytes(n, m, max_bins))
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_census: buffer too small");
  hipStream_t st = (hipStream_t)stream;
  CensusView C;
  census_layout(max_bins, n, class_capacity(n, m, 1), &C, d_census);
  int rc = fill<uint64_t>(C.table, (uint64_t)C.cap * kPairs, 0, st);
  if (rc) return rc;
  k_census_keys<<<1, 256, 0, st>>>(C, tau, omega, max_bins);
  WEDGE_LAUNCH_CHECK("k_census_keys");
  if (m == 0) return WEDGE_OK;
  IndexView ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  {
    uint64_t blocks = ceil_div(n, 256);
    if (blocks > 8192) blocks = 8192;
    k_vertex_bucket<<<(unsigned)blocks, 256, 0, st>>>(d_rowptr, n, C.vbucket);
    WEDGE_LAUNCH_CHECK("k_vertex_bucket");
  }
  k_class_work<<<1, 1024, 0, st>>>(ix, n, C.cls_work);
  WEDGE_LAUNCH_CHECK("k_class_work");
  // equal shares of the total degree 2m along the centre order
  const uint64_t total = 2 * m;
  uint64_t work = ceil_div(total, 4096);
  if (work < 4096) work = 4096;
  const uint64_t chunks = ceil_div(total, work);
  k_census<<<(unsigned)chunks, kCensusWG, 0, st>>>(d_rowptr, d_col, ix, n, work,
                                                    (uint32_t)chunks, tau, omega, max_bins, C);
  WEDGE_LAUNCH_CHECK("k_census");
  return WEDGE_OK;
}

extern "C" int wedge_cv_census_keys(const void* d_census, uint32_t max_bins, uint32_t* h_nkeys,
                                    uint32_t* h_key_bin, uint32_t* h_key_bucket, void* stream) {
  clear_error();
  if (!d_census || !h_nkeys) return set_error(WEDGE_EINVAL, "wedge_cv_census_keys: null pointer");
  CensusView C;
  census_layout(max_bins, 0, 0, &C, const_cast<void*>(d_census));
  WEDGE_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  WEDGE_HIP_TRY(hipMemcpy(h_nkeys, C.nkeys, 4, hipMemcpyDeviceToHost));
  const uint32_t nk = *h_nkeys;
  if (h_key_bin) WEDGE_HIP_TRY(hipMemcpy(h_key_bin, C.key_bin, 4 * nk, hipMemcpyDeviceToHost));
  if (h_key_bucket)
    WEDGE_HIP_TRY(hipMemcpy(h_key_bucket, C.key_bucket, 4 * nk, hipMemcpyDeviceToHost));
  return WEDGE_OK;
}

namespace wedge {
const uint32_t* census_key_of(const void* d_census, uint32_t max_bins) {
  CensusView C;
  census_layout(max_bins, 0, 0, &C, const_cast<void*>(d_census));
  return C.key_of;
}
}  // namespace wedge

extern "C" int wedge_cv_keys(void* d_census, uint32_t max_bins, uint32_t tau, uint64_t omega,
                             void* stream) {
  clear_error();
  if (!d_census || !aligned(d_census, 256))
    return set_error(WEDGE_EINVAL, "wedge_cv_keys: null or misaligned buffer");
  if (max_bins == 0 || max_bins > 4096 || tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_cv_keys: bad max_bins, tau or omega");
  CensusView C;
  census_layout(max_bins, 0, 0, &C, d_census);
  k_census_keys<<<1, 256, 0, (hipStream_t)stream>>>(C, tau, omega, max_bins);
  WEDGE_LAUNCH_CHECK("k_census_keys");
  return WEDGE_OK;
}

extern "C" size_t wedge_cv_gtable_workspace(uint32_t max_bins) {
  return round_up((uint64_t)census_cap(max_bins) * kPairs * sizeof(wedge_feature_rec), 256);
}

extern "C" int wedge_cv_gtable(const void* d_state, const void* d_census, uint32_t max_bins,
                               float* d_gtable, void* d_workspace, size_t workspace_bytes,
                               void* stream) {
  clear_error();
  if (!d_state || !d_census || !d_gtable || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_cv_gtable: null pointer");
  if (workspace_bytes < wedge_cv_gtable_workspace(max_bins))
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_gtable: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  CensusView C;
  census_layout(max_bins, 0, 0, &C, const_cast<void*>(d_census));
  uint32_t nk = 0;
  WEDGE_HIP_TRY(hipMemcpyAsync(&nk, C.nkeys, 4, hipMemcpyDeviceToHost, st));
  WEDGE_HIP_TRY(hipStreamSynchronize(st));
  if (nk > C.cap) nk = C.cap;
  const uint64_t recs = (uint64_t)nk * kPairs;
  if (recs == 0) return WEDGE_OK;
  wedge_feature_rec* rec = (wedge_feature_rec*)d_workspace;
  k_census_records<<<(unsigned)ceil_div(recs, 256), 256, 0, st>>>(C, rec);
  WEDGE_LAUNCH_CHECK("k_census_records");
  return mlp_forward_impl(d_state, rec, recs, d_gtable, st);
}

extern "C" size_t wedge_cv_exact_mean_workspace(uint32_t max_bins) {
  const uint64_t recs = (uint64_t)census_cap(max_bins) * kPairs;
  return round_up(recs * sizeof(wedge_feature_rec), 256) + round_up(recs * 4, 256);
}

extern "C" int wedge_cv_exact_mean(const void* d_state, const void* d_census, uint32_t max_bins,
                                   double* d_key_sum, uint64_t* d_key_count, void* d_workspace,
                                   size_t workspace_bytes, void* stream) {
  clear_error();
  if (!d_state || !d_census || !d_key_sum || !d_key_count || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_cv_exact_mean: null pointer");
  if (workspace_bytes < wedge_cv_exact_mean_workspace(max_bins))
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_exact_mean: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  CensusView C;
  census_layout(max_bins, 0, 0, &C, const_cast<void*>(d_census));
  const uint64_t cap_recs = (uint64_t)C.cap * kPairs;
  wedge_feature_rec* rec = (wedge_feature_rec*)d_workspace;
  float* g = (float*)((char*)d_workspace + round_up(cap_recs * sizeof(wedge_feature_rec), 256));
  // the network runs over the keys present only
  uint32_t nk = 0;
  WEDGE_HIP_TRY(hipMemcpyAsync(&nk, C.nkeys, 4, hipMemcpyDeviceToHost, st));
  WEDGE_HIP_TRY(hipStreamSynchronize(st));
  if (nk > C.cap) nk = C.cap;
  const uint64_t recs = (uint64_t)nk * kPairs;
  int rc2 = fill<double>(d_key_sum, C.cap, 0.0, st);
  if (rc2) return rc2;
  rc2 = fill<uint64_t>(d_key_count, C.cap, 0, st);
  if (rc2) return rc2;
  if (recs == 0) return WEDGE_OK;
  k_census_records<<<(unsigned)ceil_div(recs, 256), 256, 0, st>>>(C, rec);
  WEDGE_LAUNCH_CHECK("k_census_records");
  int rc = mlp_forward_impl(d_state, rec, recs, g, st);
  if (rc) return rc;
  k_census_dot<<<nk, 256, 0, st>>>(C, g, d_key_sum, d_key_count);
  WEDGE_LAUNCH_CHECK("k_census_dot");
  return WEDGE_OK;
}
