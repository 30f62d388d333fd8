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
// Work layout: a workgroup takes a chunk of the centre order (vertices by
// degree, so keys are contiguous runs), one key segment at a time; each wave
// takes one centre, builds its 256-bucket histogram in LDS from the
// neighbours' degrees, compacts the non-empty buckets and adds every bucket
// pair's count to a 64-bit LDS table of the segment (pairs of buckets < 160,
// i.e. degrees < 2^20; rarer pairs go straight to the global table).  The
// table is flushed with one global atomic per non-zero entry.
#include "common.hpp"
#include "scan.hpp"

namespace wedge {

constexpr uint32_t kBuckets = 256;
constexpr uint32_t kPairs = kBuckets * (kBuckets + 1) / 2;     // 32896
constexpr uint32_t kLdsBuckets = 160;  // degrees below 2^20
constexpr uint32_t kLdsPairs = kLdsBuckets * (kLdsBuckets + 1) / 2;  // 12880
constexpr uint32_t kCensusWG = 512;
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
  uint32_t cap;
};

inline uint32_t census_cap(uint32_t max_bins) { return kBuckets + max_bins + 1; }

static size_t census_layout(uint32_t max_bins, CensusView* v, void* base) {
  const uint32_t cap = census_cap(max_bins);
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c + off;
    off += round_up(bytes, 256);
    return (void*)p;
  };
  void* nk = take(8);
  void* ko = take((size_t)max_bins * kBuckets * 4);
  void* kb = take((size_t)cap * 4);
  void* kk = take((size_t)cap * 4);
  void* kr = take((size_t)cap * 4);
  void* tb = take((size_t)cap * kPairs * 8);
  if (v) {
    v->nkeys = (uint32_t*)nk;
    v->key_of = (uint32_t*)ko;
    v->key_bin = (uint32_t*)kb;
    v->key_bucket = (uint32_t*)kk;
    v->key_rep = (uint32_t*)kr;
    v->table = (uint64_t*)tb;
    v->cap = cap;
  }
  return off;
}

// One thread enumerates the (bin, bucket) keys that degrees >= 2 can take,
// in increasing degree order.
__global__ void k_census_keys(CensusView C, uint32_t tau, uint64_t omega, uint32_t max_bins) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  for (uint32_t i = 0; i < max_bins * kBuckets; ++i) C.key_of[i] = kNoKey;
  uint32_t nk = 0;
  for (uint32_t k = 0; k < kBuckets; ++k) {
    uint64_t lo = bucket_rep(k), hi = bucket_rep(k + 1) - 1;
    if (hi < 2) continue;
    if (lo < 2) lo = 2;
    if (hi > 0xFFFFFFFFULL) hi = 0xFFFFFFFFULL;
    if (lo > hi) continue;
    // bins spanned by degrees [lo, hi]
    uint32_t b = 0;
    while (b + 1 <= max_bins && bin_lo_deg(b + 1, tau, omega) <= lo) ++b;
    for (; b < max_bins; ++b) {
      const uint64_t blo = bin_lo_deg(b, tau, omega);
      if (blo > hi) break;
      if (nk >= C.cap) break;
      C.key_of[b * kBuckets + k] = nk;
      C.key_bin[nk] = b;
      C.key_bucket[nk] = k;
      C.key_rep[nk] = (uint32_t)(blo > lo ? blo : lo);
      ++nk;
    }
  }
  *C.nkeys = nk;
}

__device__ inline uint32_t bin_of_census(uint64_t d, uint32_t tau, uint64_t omega,
                                         uint32_t limit) {
  if (d <= tau) return d < limit ? (uint32_t)d : limit;
  uint32_t b = tau;
  uint64_t lo = tau, term = 1;
  while (b < limit) {
    uint64_t next = lo + term;
    if (next < lo) next = ~0ULL;
    if (next > d) break;
    ++b;
    lo = next;
    if (__builtin_mul_overflow(term, omega, &term)) term = ~0ULL;
  }
  return b;
}

__device__ inline uint64_t deg_at(const uint64_t* rowptr, const uint32_t* vlist, uint64_t pos) {
  const uint32_t v = vlist[pos];
  return rowptr[v + 1] - rowptr[v];
}

// key of a centre of degree d, or kNoKey (d < 2, or a bin beyond the table)
__device__ inline uint32_t key_of_degree(const CensusView& C, uint64_t d, uint32_t tau,
                                         uint64_t omega, uint32_t max_bins) {
  if (d < 2) return kNoKey;
  const uint32_t b = bin_of_census(d, tau, omega, max_bins);
  if (b >= max_bins) return kNoKey;
  return C.key_of[b * kBuckets + bucket_of(d)];
}

__global__ __launch_bounds__(kCensusWG) void k_census(const uint64_t* __restrict__ rowptr,
                                                      const uint32_t* __restrict__ col,
                                                      const uint32_t* __restrict__ vlist,
                                                      uint64_t first, uint64_t last,
                                                      uint64_t chunk, uint32_t tau,
                                                      uint64_t omega, uint32_t max_bins,
                                                      CensusView C) {
  __shared__ unsigned long long s_tab[kLdsPairs];            // 103040 B
  __shared__ uint32_t s_hist[kCensusWG / 64][kBuckets];       // 8 KB
  __shared__ uint16_t s_list[kCensusWG / 64][kBuckets];       // 4 KB
  __shared__ uint32_t s_cnt[kCensusWG / 64][kBuckets];        // 8 KB
  __shared__ uint64_t s_seg[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = kCensusWG / 64;
  const uint64_t p0 = first + (uint64_t)blockIdx.x * chunk;
  const uint64_t p1 = min(p0 + chunk, last);
  if (p0 >= p1) return;
  for (uint32_t i = tid; i < kLdsPairs; i += kCensusWG) s_tab[i] = 0;
  for (uint32_t i = tid; i < (uint32_t)nw * kBuckets; i += kCensusWG) (&s_hist[0][0])[i] = 0;
  __syncthreads();
  uint64_t seg = p0;
  while (seg < p1) {
    if (tid == 0) {
      const uint32_t key0 = key_of_degree(C, deg_at(rowptr, vlist, seg), tau, omega, max_bins);
      // end of the run of this key: keys are monotone in the degree
      uint64_t lo = seg + 1, hi = p1;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const uint32_t km = key_of_degree(C, deg_at(rowptr, vlist, mid), tau, omega, max_bins);
        if (km == key0) lo = mid + 1; else hi = mid;
      }
      s_seg[0] = lo;
      s_seg[1] = key0;
    }
    __syncthreads();
    const uint64_t seg_end = s_seg[0];
    const uint32_t key = (uint32_t)s_seg[1];
    __syncthreads();
    if (key == kNoKey || key >= *C.nkeys) {  // centres without wedges (or beyond the bins)
      seg = seg_end;
      continue;
    }
    uint64_t* gtab = C.table + (uint64_t)key * kPairs;
    for (uint64_t pos = seg + wave; pos < seg_end; pos += nw) {
      const uint32_t v = vlist[pos];
      const uint64_t r0 = rowptr[v], r1 = rowptr[v + 1];
      for (uint64_t x = r0 + lane; x < r1; x += 64) {
        const uint32_t a = col[x];
        atomicAdd(&s_hist[wave][bucket_of(rowptr[a + 1] - rowptr[a])], 1u);
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
      uint32_t pre = nz;  // inclusive scan of nz over the wave
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
        s_hist[wave][lane * 4 + t] = 0;
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0);
      // every pair (i <= j) of non-empty buckets
      const uint32_t np = u * (u + 1) / 2;
      for (uint32_t t = lane; t < np; t += 64) {
        uint32_t j = (uint32_t)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (j * (j + 1) / 2 > t) --j;
        while ((j + 1) * (j + 2) / 2 <= t) ++j;
        const uint32_t i = t - j * (j + 1) / 2;
        const uint64_t hi_ = s_cnt[wave][i], hj = s_cnt[wave][j];
        const uint64_t cnt = (i == j) ? hi_ * (hi_ - 1) / 2 : hi_ * hj;
        if (cnt == 0) continue;
        const uint32_t bi = s_list[wave][i], bj = s_list[wave][j];
        if (bj < kLdsBuckets)
          atomicAdd(&s_tab[pair_index(bi, bj)], (unsigned long long)cnt);
        else
          atomicAdd((unsigned long long*)&gtab[pair_index(bi, bj)], (unsigned long long)cnt);
      }
      __builtin_amdgcn_wave_barrier();
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

extern "C" size_t wedge_cv_census_bytes(uint32_t max_bins) {
  return census_layout(max_bins, nullptr, nullptr);
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
  if (census_bytes < census_layout(max_bins, nullptr, nullptr))
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_census: buffer too small");
  hipStream_t st = (hipStream_t)stream;
  CensusView C;
  census_layout(max_bins, &C, d_census);
  int rc = fill<uint64_t>(C.table, (uint64_t)C.cap * kPairs, 0, st);
  if (rc) return rc;
  k_census_keys<<<1, 1, 0, st>>>(C, tau, omega, max_bins);
  WEDGE_LAUNCH_CHECK("k_census_keys");
  if (m == 0) return WEDGE_OK;
  IndexView ix = index_view(const_cast<void*>(d_index), n, m, 1, max_bins);
  // every position of the centre order; runs of degree 0 and 1 are skipped
  const uint64_t chunk = 2048;
  const uint64_t blocks = ceil_div(n, chunk);
  k_census<<<(unsigned)blocks, kCensusWG, 0, st>>>(d_rowptr, d_col, ix.vlist, 0, n, chunk, tau,
                                                    omega, max_bins, C);
  WEDGE_LAUNCH_CHECK("k_census");
  return WEDGE_OK;
}

extern "C" int wedge_cv_census_keys(const void* d_census, uint32_t max_bins, uint32_t* h_nkeys,
                                    uint32_t* h_key_bin, uint32_t* h_key_bucket, void* stream) {
  clear_error();
  if (!d_census || !h_nkeys) return set_error(WEDGE_EINVAL, "wedge_cv_census_keys: null pointer");
  CensusView C;
  census_layout(max_bins, &C, const_cast<void*>(d_census));
  WEDGE_HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  WEDGE_HIP_TRY(hipMemcpy(h_nkeys, C.nkeys, 4, hipMemcpyDeviceToHost));
  const uint32_t nk = *h_nkeys;
  if (h_key_bin) WEDGE_HIP_TRY(hipMemcpy(h_key_bin, C.key_bin, 4 * nk, hipMemcpyDeviceToHost));
  if (h_key_bucket)
    WEDGE_HIP_TRY(hipMemcpy(h_key_bucket, C.key_bucket, 4 * nk, hipMemcpyDeviceToHost));
  return WEDGE_OK;
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
  census_layout(max_bins, &C, const_cast<void*>(d_census));
  const uint64_t recs = (uint64_t)C.cap * kPairs;
  wedge_feature_rec* rec = (wedge_feature_rec*)d_workspace;
  float* g = (float*)((char*)d_workspace + round_up(recs * sizeof(wedge_feature_rec), 256));
  k_census_records<<<(unsigned)ceil_div(recs, 256), 256, 0, st>>>(C, rec);
  WEDGE_LAUNCH_CHECK("k_census_records");
  int rc = mlp_forward_impl(d_state, rec, recs, g, st);
  if (rc) return rc;
  int rc2 = fill<double>(d_key_sum, C.cap, 0.0, st);
  if (rc2) return rc2;
  rc2 = fill<uint64_t>(d_key_count, C.cap, 0, st);
  if (rc2) return rc2;
  k_census_dot<<<C.cap, 256, 0, st>>>(C, g, d_key_sum, d_key_count);
  WEDGE_LAUNCH_CHECK("k_census_dot");
  return WEDGE_OK;
}
