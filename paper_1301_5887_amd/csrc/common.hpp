// Shared host/device helpers of libwedge: status plumbing, launch checks and
// the index layout that wedge_bin_counts writes and wedge_sample_close reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/wedge.h"

namespace wedge {

// Thread-local last-error message; set_error returns the status so callers
// can `return set_error(...)`.
int set_error(int status, const char* fmt, ...);
void clear_error();

#define WEDGE_HIP_TRY(expr)                                                        \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return ::wedge::set_error(WEDGE_EHIP, "%s failed: %s (%s:%d)", #expr,       \
                                hipGetErrorString(_e), __FILE__, __LINE__);        \
  } while (0)

#define WEDGE_LAUNCH_CHECK(what)                                                   \
  do {                                                                             \
    hipError_t _e = hipGetLastError();                                             \
    if (_e != hipSuccess)                                                          \
      return ::wedge::set_error(WEDGE_EHIP, "launch of %s failed: %s", what,       \
                                hipGetErrorString(_e));                            \
  } while (0)

inline bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Number of significant bits of x (0 for x == 0).
inline int bit_width(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// ---------------------------------------------------------------- the index
// Device blob written by wedge_bin_counts.  All sections 256-byte aligned.
struct IndexHeader {
  uint32_t n;
  uint32_t max_bins;
  uint32_t num_classes;   // distinct degrees present (degree 0 included)
  uint32_t tau;
  uint64_t omega;
  uint64_t class_cap;
  uint64_t overflow;      // vertices whose bin is >= max_bins
  uint64_t empty_bin_samples;  // samples asked of a bin with p_b = 0
  uint64_t mismatch;      // sampler launches whose n / max_bins / m disagree
  uint32_t num_graphs;
  uint32_t pad32;
  uint64_t pad[24];
};
static_assert(sizeof(IndexHeader) == 256, "header is one 256-byte line");

// One row per bin b < max_bins plus row max_bins for the global stream.
struct BinMeta {
  uint64_t lo_deg;     // BinLoDeg(b); row max_bins: 2 (all d >= 2)
  uint64_t hi_deg;     // BinLoDeg(b+1), exclusive; row max_bins: 2^64-1
  uint64_t n_b;
  uint64_t p_b;        // wedges in the bin
  uint64_t cumw_base;  // wedges of all classes before cls_lo
  uint32_t cls_lo;     // classes of the bin: [cls_lo, cls_hi)
  uint32_t cls_hi;
  uint64_t pad[2];
};
static_assert(sizeof(BinMeta) == 64, "bin row is 64 bytes");

struct IndexView {
  IndexHeader* hdr;
  BinMeta* bins;      // [max_bins + 1]
  uint32_t* vlist;    // [n] vertices ordered by (degree, id)
  uint64_t* vrow;     // [n] rowptr[vlist[i]]: adjacency start of each centre
  uint32_t* cls_deg;  // [class_cap] degree of class j (ascending)
  uint32_t* cls_start;// [class_cap] first position of class j in vlist
  uint64_t* cls_cumw; // [class_cap] inclusive prefix of count_j * C(d_j, 2)
  uint8_t* vcode;     // [n] degree code floor(8 L(d)) per vertex id (monotone in d)
  uint64_t* vmeta;    // [n+1] rowptr[v] | code(v) << 56 (row start and degree code)
};

constexpr uint64_t kRowMask = (1ULL << 56) - 1;

// Upper bound on the number of distinct (graph, degree) pairs of G simple
// graphs with n_total vertices and m_total edges in all.
uint64_t class_capacity(uint64_t n_total, uint64_t m_total, uint32_t G);
size_t index_bytes(uint64_t n_total, uint64_t m_total, uint32_t G, uint32_t max_bins);
IndexView index_view(void* base, uint64_t n_total, uint64_t m_total, uint32_t G,
                     uint32_t max_bins);

// Sampling index of G graphs whose vertices are the consecutive global id
// ranges [voff[g], voff[g+1]) of one block-diagonal CSR (d_voff may be null
// when G == 1); degrees must be < 2^(32 - bits(G-1)).  Rows of the index:
// G x (max_bins + 1), row max_bins of a graph being its global stream.
size_t bins_workspace_bytes(uint64_t n_total, uint32_t G, uint32_t max_bins);
int bins_build(const uint64_t* d_rowptr, uint64_t n, uint64_t m_total, const uint32_t* d_voff,
               uint32_t G, uint32_t max_n, uint32_t tau, uint64_t omega, uint32_t max_bins,
               uint64_t* d_n_b, uint64_t* d_p_b, void* d_index, void* d_workspace,
               hipStream_t st);

// Block-diagonal CSR of G graphs (G == 1: d_eoff, d_voff may be null):
// edges [eoff[g], eoff[g+1]) of the input carry local ids of graph g, whose
// global ids are voff[g] + local.
size_t csr_workspace_bytes(uint64_t m_in);
// Device check of an adjacency (validate.hip); validate_or_fail also waits
// for it and returns WEDGE_EGRAPH when it finds a fault.
int validate_csr(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                 uint64_t* d_counts, hipStream_t st);
bool validate_requested();
int validate_or_fail(const char* who, const uint64_t* d_rowptr, const uint32_t* d_col,
                     uint32_t n, uint64_t m, uint64_t* d_counts, hipStream_t st);

int csr_build(const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_in, uint32_t n,
              const uint64_t* d_eoff, const uint32_t* d_voff, uint32_t G, uint64_t* d_rowptr,
              uint32_t* d_col, uint64_t* d_info, void* d_workspace, hipStream_t st);

// Forward pass of the control-variate network (mlp.hip).
int mlp_forward_impl(const void* d_state, const wedge_feature_rec* d_x, uint64_t n, float* d_g,
                     hipStream_t st);

// Graph of global vertex v: last g with voff[g] <= v (voff[0] = 0).
__device__ inline uint32_t graph_of(const uint32_t* __restrict__ voff, uint32_t G, uint32_t v) {
  if (G <= 1) return 0;
  uint32_t lo = 0, hi = G;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (voff[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// Saturating BinLoDeg (host and device).
__host__ __device__ inline uint64_t bin_lo_deg(uint32_t b, uint32_t tau, uint64_t omega) {
  if (b <= tau) return b;
  uint64_t lo = tau, term = 1;
  for (uint32_t j = 0; j + tau < b; ++j) {
    uint64_t nlo = lo + term;
    if (nlo < lo) return ~0ULL;
    lo = nlo;
    uint64_t hi = __builtin_mul_overflow(term, omega, &term) ? 1 : 0;
    if (hi) term = ~0ULL;
  }
  return lo;
}

// BinId(d) of the integer reading of Eq. binid for d >= 1 (the largest b
// with BinLoDeg(b) <= d), or `limit` when that bin would be >= limit.
__host__ __device__ inline uint32_t bin_id_capped(uint64_t d, uint32_t tau, uint64_t omega,
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

// Key id of every (bin, centre bucket) in a census buffer ([max_bins][256]
// uint32, 0xFFFFFFFF where degrees >= 2 cannot take the pair).
const uint32_t* census_key_of(const void* d_census, uint32_t max_bins);

}  // namespace wedge
