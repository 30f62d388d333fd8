// CPU oracle for wedge sampling of triangle statistics.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file.  Only tests, the smoke check and the CPU-baseline leg of
// the benchmark use it.  It shares no code with the HIP path: it has its own
// Philox, its own uniform-below, its own binning and a different search
// structure (a per-vertex prefix array and one global sorted edge-key array
// instead of the GPU's degree-class table and per-row search).
//
// Method: Kolda, Pinar, Plantenga, Seshadhri, Task, "Counting Triangles in
// Massive Graphs with MapReduce" (arXiv 1301.5887).
//   Sec. 2.1        degrees, wedges p_i = C(d_i,2), closed wedges, c = 3t/p
//   Sec. 2.2        binned quantities W_{D,q}, c_D, t_D
//   Sec. 3.1        Hoeffding sample size (Thm "Hoeffding")
//   Sec. 3.2        binned estimators (Thms "cd-est", "td-est"), choosing
//                   uniform random wedges (center with prob p_i/p_D, then two
//                   distinct neighbours)
//   Sec. 4.2        BinLoDeg / BinId (Eqs. binlodeg, binid)
//   Alg. phase3b    exact closure test (either orientation of the edge)
//   Alg. phase4c    per-bin classes q0..q3 and the summary c, t
//   Eq. global_est  global estimate from the bins
//
// Readings where the paper is silent or garbled (all listed in the design
// notes): integer BinLoDeg/BinId for integer omega >= 2; c_D divides by p_D;
// neighbours numbered in ascending id order; centres of a bin ordered by
// (degree, id); Philox4x64-10 keyed by (seed, domain) with counter
// (sample, bin, graph, retry round); Lemire's nearly-divisionless method for
// uniform integers; exactly k i.i.d. samples per non-empty bin.
//
// Parity pins: every exported function is checked by the CPU tests against
// values fixed outside this file (the worked example of Sec. 2.2, closed
// forms, identities, numpy's Philox, exhaustive uniform-below at 16 bits,
// brute-force enumeration in pure Python, chi-square uniformity).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#include <parallel/algorithm>
#endif

typedef unsigned __int128 u128;

namespace {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11).  Two 64x64->128 multiplies per round, a Weyl key
// schedule, ten rounds.
// ---------------------------------------------------------------------------
const uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ULL;
const uint64_t kPhiloxM1 = 0xCA5A826395121157ULL;
const uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ULL;
const uint64_t kPhiloxW1 = 0xBB67AE8584CAA73BULL;

void philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    u128 p0 = (u128)kPhiloxM0 * c0;
    u128 p1 = (u128)kPhiloxM1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Key domains (the key's second word): 1 = plain sampling; 2, 3, 4 = the
// training, auxiliary and evaluation streams of the control variate.
const uint64_t kDomainSample = 1;
const uint64_t kGlobalBin = 0xFFFFFFFFULL;  // counter word 1 of the global stream

// ---------------------------------------------------------------------------
// Uniform integer on [0, N) by Lemire's nearly-divisionless method (Lemire,
// "Fast random integer generation in an interval", ACM TOMACS 2019).  Written
// once for any word width so that the 16-bit instance can be checked
// exhaustively and the 64-bit instance is the same code.
// `next()` returns the word of retry round 0, 1, 2, ... in order.
// ---------------------------------------------------------------------------
template <class Word, class Wide, class Source>
Word lemire_below(Word N, Source& next) {
  const int bits = 8 * (int)sizeof(Word);
  Word x = next();
  Wide m = (Wide)x * (Wide)N;
  Word l = (Word)m;
  if (l < N) {
    Word thr = (Word)((Word)(0 - N) % N);  // 2^bits mod N
    while (l < thr) {
      x = next();
      m = (Wide)x * (Wide)N;
      l = (Word)m;
    }
  }
  return (Word)(m >> bits);
}

// One of the two random draws of a sample: word `t` of Philox blocks with
// counters (s, b, g, r) for r = 0, 1, 2, ...
struct PhiloxWord {
  uint64_t key[2];
  uint64_t ctr[4];
  int t;
  uint64_t operator()() {
    uint64_t out[4];
    philox(ctr, key, out);
    ctr[3] += 1;  // next retry round
    return out[t];
  }
};

uint64_t draw_below(uint64_t seed, uint64_t domain, uint64_t s, uint64_t bin_word,
                    uint64_t graph, int t, uint64_t N) {
  PhiloxWord src;
  src.key[0] = seed;
  src.key[1] = domain;
  src.ctr[0] = s;
  src.ctr[1] = bin_word;
  src.ctr[2] = graph;
  src.ctr[3] = 0;
  src.t = t;
  return lemire_below<uint64_t, u128>(N, src);
}

// ---------------------------------------------------------------------------
// Binning, Sec. 4.2, integer reading: BinLoDeg(b) = b for b <= tau, else
// tau + sum_{j=0}^{b-tau-1} omega^j (saturating at 2^64-1);
// BinId(d) = max{ b : BinLoDeg(b) <= d } for d >= 1.
// ---------------------------------------------------------------------------
uint64_t bin_lo_deg(uint32_t b, uint32_t tau, uint64_t omega) {
  if (b <= tau) return b;
  u128 lo = tau;
  u128 term = 1;
  const u128 cap = ~(uint64_t)0;
  for (uint32_t j = 0; j + tau < b; ++j) {
    lo += term;
    if (lo >= cap) return ~(uint64_t)0;
    term *= omega;
    if (term > cap) term = cap;
  }
  return (uint64_t)lo;
}

uint32_t bin_id(uint64_t d, uint32_t tau, uint64_t omega) {
  // Linear walk up from bin 0: plain and obviously the definition.
  uint32_t b = 0;
  while (bin_lo_deg(b + 1, tau, omega) <= d) {
    ++b;
    if (b > 100000) break;
  }
  return b;
}

// BinId for many vertices: max{ b < nb : BinLoDeg(b) <= d } read off a table
// of BinLoDeg(0..nb).  Returns nb when d >= BinLoDeg(nb) (out of range).
struct BinTable {
  std::vector<uint64_t> lo;
  uint32_t nb;
  BinTable(uint32_t tau, uint64_t omega, uint32_t nbins) : nb(nbins) {
    for (uint32_t b = 0; b <= nbins; ++b) lo.push_back(bin_lo_deg(b, tau, omega));
  }
  uint32_t operator()(uint64_t d) const {
    size_t j = (size_t)(std::upper_bound(lo.begin(), lo.end(), d) - lo.begin());
    return (uint32_t)(j - 1);  // lo[0] = 0 <= d, so j >= 1
  }
};

inline uint64_t choose2(uint64_t d) { return d < 2 ? 0 : d * (d - 1) / 2; }

// (degree, id) pairs in ascending order: the centre order of a bin.
inline void psort(std::vector<std::pair<uint64_t, uint32_t>>& dv) {
#ifdef _OPENMP
  __gnu_parallel::sort(dv.begin(), dv.end());
#else
  std::sort(dv.begin(), dv.end());
#endif
}

inline bool has_edge(const uint64_t* keys, uint64_t m, uint32_t a, uint32_t c) {
  uint32_t lo = a < c ? a : c, hi = a < c ? c : a;
  uint64_t key = ((uint64_t)lo << 32) | hi;
  return std::binary_search(keys, keys + m, key);
}

}  // namespace

extern "C" {

// Threads an OpenMP region of the oracle uses (1 without OpenMP).
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Sets the thread count of the oracle's later parallel regions (and of
// any other OpenMP code in the process).
void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

// -------------------------------------------------------------- primitives
void orc_philox4x64_10(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  philox(ctr, key, out);
}

// 16-bit instance of the uniform-below method.  `xs` is the sequence of
// words returned by successive retry rounds; `*consumed` receives how many
// were used.  Used only to check the method exhaustively.
uint32_t orc_lemire16(uint32_t N, const uint16_t* xs, int nx, int* consumed) {
  struct Seq {
    const uint16_t* xs;
    int nx, pos;
    uint16_t operator()() { return pos < nx ? xs[pos++] : (pos++, (uint16_t)0xFFFF); }
  } seq{xs, nx, 0};
  uint16_t r = lemire_below<uint16_t, uint32_t>((uint16_t)N, seq);
  *consumed = seq.pos;
  return r;
}

// 64-bit instance with an explicit word sequence (checks the retry path).
uint64_t orc_lemire64_seq(uint64_t N, const uint64_t* xs, int nx, int* consumed) {
  struct Seq {
    const uint64_t* xs;
    int nx, pos;
    uint64_t operator()() { return pos < nx ? xs[pos++] : (pos++, ~(uint64_t)0); }
  } seq{xs, nx, 0};
  uint64_t r = lemire_below<uint64_t, u128>(N, seq);
  *consumed = seq.pos;
  return r;
}

// The draw the sampler uses: word t of Philox((seed,1), (s, bin_word, g, r)).
uint64_t orc_draw_below(uint64_t seed, uint64_t s, uint64_t bin_word, uint64_t graph, int t,
                        uint64_t N) {
  return draw_below(seed, kDomainSample, s, bin_word, graph, t, N);
}

uint64_t orc_bin_lo_deg(uint32_t b, uint32_t tau, uint64_t omega) { return bin_lo_deg(b, tau, omega); }
uint32_t orc_bin_id(uint64_t d, uint32_t tau, uint64_t omega) { return bin_id(d, tau, omega); }

// Thm "Hoeffding": k = ceil(0.5 eps^-2 ln(2/delta)), in double with libm log.
uint64_t orc_hoeffding_k(double eps, double delta) {
  double k = 0.5 / (eps * eps) * std::log(2.0 / delta);
  return (uint64_t)std::ceil(k);
}

// ------------------------------------------------------------ graph set-up
// Canonical edge set (Sec. 4.1 input convention; Sec. 5.1 "treated as
// undirected"): drop self-loops, store (min, max) as key min<<32|max, sort,
// remove duplicates.  Edges with an id >= n are rejected and counted.
// Returns m; keys_out must hold m_in entries.  Dropped edges first take the
// value 2^64-1, which no kept key can have (its low word would be an id
// >= 2^32-1 > max), so after the sort they sit at the end and are cut off.
uint64_t orc_canon(const uint32_t* src, const uint32_t* dst, uint64_t m_in, uint32_t n,
                   uint64_t* keys_out, uint64_t* rejected) {
  const uint64_t kDropped = ~(uint64_t)0;
  uint64_t rej = 0;
#pragma omp parallel for schedule(static) reduction(+ : rej)
  for (int64_t i = 0; i < (int64_t)m_in; ++i) {
    uint32_t u = src[i], w = dst[i];
    if (u >= n || w >= n) { ++rej; keys_out[i] = kDropped; continue; }
    if (u == w) { keys_out[i] = kDropped; continue; }
    uint32_t lo = u < w ? u : w, hi = u < w ? w : u;
    keys_out[i] = ((uint64_t)lo << 32) | hi;
  }
#ifdef _OPENMP
  __gnu_parallel::sort(keys_out, keys_out + m_in);
#else
  std::sort(keys_out, keys_out + m_in);
#endif
  uint64_t cnt = (uint64_t)(std::lower_bound(keys_out, keys_out + m_in, kDropped) - keys_out);
  uint64_t m = (uint64_t)(std::unique(keys_out, keys_out + cnt) - keys_out);
  if (rejected) *rejected = rej;
  return m;
}

// Adjacency lists from canonical keys: N(v) holds every neighbour once, in
// ascending id order.  rowptr[n+1], col[2m].  Rows are filled in any order
// (parallel) and then each row is sorted, so the result is the definition's.
void orc_csr(const uint64_t* keys, uint64_t m, uint32_t n, uint64_t* rowptr, uint32_t* col) {
  std::vector<uint64_t> deg(n, 0);
  uint64_t* dg = deg.data();
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) {
    __atomic_fetch_add(&dg[(uint32_t)(keys[e] >> 32)], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&dg[(uint32_t)keys[e]], 1, __ATOMIC_RELAXED);
  }
  rowptr[0] = 0;
  for (uint32_t v = 0; v < n; ++v) rowptr[v + 1] = rowptr[v] + deg[v];
  std::vector<uint64_t> fill(rowptr, rowptr + n);
  uint64_t* fl = fill.data();
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)m; ++e) {
    uint32_t a = (uint32_t)(keys[e] >> 32), b = (uint32_t)keys[e];
    col[__atomic_fetch_add(&fl[a], 1, __ATOMIC_RELAXED)] = b;
    col[__atomic_fetch_add(&fl[b], 1, __ATOMIC_RELAXED)] = a;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t v = 0; v < (int64_t)n; ++v) std::sort(col + rowptr[v], col + rowptr[v + 1]);
}

// Phase 1b: per bin b, n_b = #vertices, p_b = sum of C(d,2).  Degree-0
// vertices are in no bin.  Returns 0, or -2 if some degree has BinId >= max_bins.
int orc_bins(const uint64_t* rowptr, uint32_t n, uint32_t tau, uint64_t omega, uint32_t max_bins,
             uint64_t* n_b, uint64_t* p_b) {
  for (uint32_t b = 0; b < max_bins; ++b) n_b[b] = p_b[b] = 0;
  BinTable bins(tau, omega, max_bins);
  int out_of_range = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_b[:max_bins], p_b[:max_bins]) \
    reduction(| : out_of_range)
  for (int64_t v = 0; v < (int64_t)n; ++v) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    if (d == 0) continue;
    uint32_t b = bins(d);
    if (b >= max_bins) { out_of_range = 1; continue; }
    n_b[b] += 1;
    p_b[b] += choose2(d);
  }
  return out_of_range ? -2 : 0;
}

// The centre order of the global stream: every vertex with d >= 2, sorted
// by (degree, id).  Returns the count written to order_out[n].
uint64_t orc_center_order(const uint64_t* rowptr, uint32_t n, uint32_t* order_out) {
  std::vector<std::pair<uint64_t, uint32_t>> dv;
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    if (d >= 2) dv.push_back({d, v});
  }
  psort(dv);
  for (size_t i = 0; i < dv.size(); ++i) order_out[i] = dv[i].second;
  return dv.size();
}

// ------------------------------------------------------------ sampling mode
// Thm "cd-est"/"td-est" with the centre-then-pair construction of Sec. 3.2.
// For every bin b < max_bins with k_per_bin[b] > 0 (the caller passes 0 for
// bins without wedges) draw samples s = 0..k_b-1:
//   w  = U(word 0, p_b); centre v = L_b[first j with P_b[j] > w]
//   o  = U(word 1, d(d-1)); i = o / (d-1); r = o mod (d-1); j = r + [r >= i]
//   a  = N(v)[i], c = N(v)[j]; closed = {a,c} in E
//   cls = 0 if open, else 1 + [BinId(d_a) = b] + [BinId(d_c) = b]
// and the global stream (one bin of all d >= 2, counter word 1 = 2^32-1):
// cls = 3 if closed (both endpoints then have d >= 2), else 0.
// q[(max_bins+1)*4]: row max_bins is the global stream.
// Samples s run over [s_begin, s_begin + k) with Philox key (seed, domain).
// Dump (nullable): for bin row r and s - s_begin < dump_per_bin, entry
// r*dump_per_bin + (s - s_begin) of v/a/c/cls.  Returns 0, -1 on bad input.
int orc_sample(const uint64_t* rowptr, const uint32_t* col, uint32_t n, const uint64_t* keys,
               uint64_t m, uint32_t tau, uint64_t omega, uint32_t max_bins,
               const uint64_t* k_per_bin, uint64_t k_global, uint64_t seed, uint32_t graph_id,
               uint64_t domain, uint64_t s_begin, uint64_t* q, uint32_t* dump_v,
               uint32_t* dump_a, uint32_t* dump_c, uint8_t* dump_cls, uint64_t dump_per_bin,
               int nthreads) {
  for (uint64_t i = 0; i < (uint64_t)(max_bins + 1) * 4; ++i) q[i] = 0;
  // per-vertex degree and bin
  std::vector<uint64_t> deg(n);
  std::vector<uint32_t> vbin(n, 0);
  BinTable bins(tau, omega, max_bins);
  int out_of_range = 0;
#pragma omp parallel for schedule(static) reduction(| : out_of_range)
  for (int64_t v = 0; v < (int64_t)n; ++v) {
    deg[v] = rowptr[v + 1] - rowptr[v];
    if (deg[v] == 0) continue;
    uint32_t b = bins(deg[v]);
    if (b >= max_bins) out_of_range = 1;
    vbin[v] = b;
  }
  if (out_of_range) return -1;
  // L_b lists ordered by (d, id) and their inclusive prefix sums of p_v.
  std::vector<uint32_t> order;
  {
    std::vector<std::pair<uint64_t, uint32_t>> dv;
    for (uint32_t v = 0; v < n; ++v)
      if (deg[v] >= 2) dv.push_back({deg[v], v});
    psort(dv);
    order.resize(dv.size());
    for (size_t i = 0; i < dv.size(); ++i) order[i] = dv[i].second;
  }
  std::vector<std::vector<uint32_t>> L(max_bins + 1);
  std::vector<std::vector<uint64_t>> P(max_bins + 1);
  for (uint32_t v : order) {
    uint32_t b = vbin[v];
    L[b].push_back(v);
    P[b].push_back((P[b].empty() ? 0 : P[b].back()) + choose2(deg[v]));
    L[max_bins].push_back(v);
    P[max_bins].push_back((P[max_bins].empty() ? 0 : P[max_bins].back()) + choose2(deg[v]));
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int bad = 0;
  for (uint32_t row = 0; row <= max_bins; ++row) {
    const bool global = (row == max_bins);
    const uint64_t k = global ? k_global : k_per_bin[row];
    if (k == 0) continue;
    if (L[row].empty()) { bad = 1; continue; }  // samples asked of a bin without wedges
    const uint64_t pb = P[row].back();
    const uint64_t bin_word = global ? kGlobalBin : row;
    const uint32_t* Lr = L[row].data();
    const uint64_t* Pr = P[row].data();
    const size_t nL = L[row].size();
    uint64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
#pragma omp parallel for schedule(static) reduction(+ : c0, c1, c2, c3)
    for (int64_t si = 0; si < (int64_t)k; ++si) {
      const uint64_t s = s_begin + (uint64_t)si;
      uint64_t w = draw_below(seed, domain, s, bin_word, graph_id, 0, pb);
      size_t j = (size_t)(std::upper_bound(Pr, Pr + nL, w) - Pr);
      uint32_t v = Lr[j];
      uint64_t d = deg[v];
      uint64_t o = draw_below(seed, domain, s, bin_word, graph_id, 1, d * (d - 1));
      uint64_t i = o / (d - 1);
      uint64_t r = o % (d - 1);
      uint64_t j2 = r + (r >= i ? 1 : 0);
      uint32_t a = col[rowptr[v] + i];
      uint32_t c = col[rowptr[v] + j2];
      bool closed = has_edge(keys, m, a, c);
      uint8_t cls = 0;
      if (closed) {
        if (global)
          cls = 3;
        else
          cls = (uint8_t)(1 + (vbin[a] == row ? 1 : 0) + (vbin[c] == row ? 1 : 0));
      }
      if (cls == 0) ++c0; else if (cls == 1) ++c1; else if (cls == 2) ++c2; else ++c3;
      if (dump_v && (uint64_t)si < dump_per_bin) {
        uint64_t at = (uint64_t)row * dump_per_bin + (uint64_t)si;
        dump_v[at] = v;
        dump_a[at] = a;
        dump_c[at] = c;
        dump_cls[at] = cls;
      }
    }
    q[row * 4 + 0] = c0;
    q[row * 4 + 1] = c1;
    q[row * 4 + 2] = c2;
    q[row * 4 + 3] = c3;
  }
  return bad ? -1 : 0;
}

// ------------------------------------------------- Phase 2a allocation mode
// Alg. phase2a then the Sampling procedure of Alg. phase2c: every vertex v of
// a row (bin b, or the whole graph for the global row) with d >= 2 gets
// q_v = floor(q*) or ceil(q*) samples, q* = C(d,2) k / p_row, ceil with
// probability q* - floor(q*) exactly (so E[q_v] = q*); the printed test
// "x >= frac ? ceil : floor" would give ceil with probability 1 - frac, which
// contradicts the text's example, so the text is followed).  The rounding draw
// of v is uniform on [0, p_row) from word 2 of Philox blocks (v, b, g, r) and
// rounds up iff it is below (C(d,2) k) mod p_row.  Samples are numbered s = 0,
// 1, ... through the row's vertices in (degree, id) order; sample s at v takes
// its ordered neighbour pair from word 1 of blocks (s, b, g, r), as the
// i.i.d. sampler does.  Key (seed, domain).  Outputs: q[row][4] class counts,
// totals[row] = sum of q_v, and the first dump_per_bin samples of each row.
int orc_sample_alloc(const uint64_t* rowptr, const uint32_t* col, uint32_t n,
                     const uint64_t* keys, uint64_t m, uint32_t tau, uint64_t omega,
                     uint32_t max_bins, const uint64_t* k_per_bin, uint64_t k_global,
                     uint64_t seed, uint32_t graph_id, uint64_t domain, uint64_t* q,
                     uint64_t* totals, uint32_t* dump_v, uint32_t* dump_a, uint32_t* dump_c,
                     uint8_t* dump_cls, uint64_t dump_per_bin) {
  for (uint64_t i = 0; i < (uint64_t)(max_bins + 1) * 4; ++i) q[i] = 0;
  for (uint32_t r = 0; r <= max_bins; ++r) totals[r] = 0;
  std::vector<uint64_t> deg(n);
  std::vector<uint32_t> vbin(n, 0);
  BinTable bins(tau, omega, max_bins);
  for (uint32_t v = 0; v < n; ++v) {
    deg[v] = rowptr[v + 1] - rowptr[v];
    if (deg[v] == 0) continue;
    uint32_t b = bins(deg[v]);
    if (b >= max_bins) return -1;
    vbin[v] = b;
  }
  std::vector<std::pair<uint64_t, uint32_t>> dv;
  for (uint32_t v = 0; v < n; ++v)
    if (deg[v] >= 2) dv.push_back({deg[v], v});
  psort(dv);
  std::vector<std::vector<uint32_t>> L(max_bins + 1);
  std::vector<uint64_t> pb(max_bins + 1, 0);
  for (auto& e : dv) {
    L[vbin[e.second]].push_back(e.second);
    L[max_bins].push_back(e.second);
    pb[vbin[e.second]] += choose2(e.first);
    pb[max_bins] += choose2(e.first);
  }
  int bad = 0;
  for (uint32_t row = 0; row <= max_bins; ++row) {
    const bool global = (row == max_bins);
    const uint64_t k = global ? k_global : k_per_bin[row];
    if (k == 0) continue;
    if (L[row].empty()) { bad = 1; continue; }
    const uint64_t bin_word = global ? kGlobalBin : row;
    const uint64_t p = pb[row];
    uint64_t s = 0;
    for (uint32_t v : L[row]) {
      const u128 num = (u128)choose2(deg[v]) * k;
      uint64_t qv = (uint64_t)(num / p);
      const uint64_t rem = (uint64_t)(num % p);
      if (draw_below(seed, domain, v, bin_word, graph_id, 2, p) < rem) ++qv;
      const uint64_t d = deg[v];
      for (uint64_t j = 0; j < qv; ++j, ++s) {
        uint64_t o = draw_below(seed, domain, s, bin_word, graph_id, 1, d * (d - 1));
        uint64_t i = o / (d - 1);
        uint64_t r = o % (d - 1);
        uint64_t j2 = r + (r >= i ? 1 : 0);
        uint32_t a = col[rowptr[v] + i];
        uint32_t c = col[rowptr[v] + j2];
        uint8_t cls = 0;
        if (has_edge(keys, m, a, c))
          cls = global ? 3 : (uint8_t)(1 + (vbin[a] == row ? 1 : 0) + (vbin[c] == row ? 1 : 0));
        q[row * 4 + cls] += 1;
        if (dump_v && s < dump_per_bin) {
          uint64_t at = (uint64_t)row * dump_per_bin + s;
          dump_v[at] = v;
          dump_a[at] = a;
          dump_c[at] = c;
          dump_cls[at] = cls;
        }
      }
    }
    totals[row] = s;
  }
  return bad ? -1 : 0;
}

// --------------------------------------------------------------- exact mode
// Definitions of Sec. 2.1/2.2 by enumeration: for every centre v and every
// pair of distinct neighbours {a, c}, the wedge is closed iff {a,c} in E.
// P[b*4 + q] = |W_{b,q}| with q = 0 open, q = 1..3 closed with q vertices in
// bin b.  Row max_bins: global (q0 = open, q3 = closed).
int orc_exact(const uint64_t* rowptr, const uint32_t* col, uint32_t n, const uint64_t* keys,
              uint64_t m, uint32_t tau, uint64_t omega, uint32_t max_bins, uint64_t* P) {
  for (uint64_t i = 0; i < (uint64_t)(max_bins + 1) * 4; ++i) P[i] = 0;
  std::vector<uint32_t> vbin(n, 0);
  BinTable bins(tau, omega, max_bins);
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    if (d == 0) continue;
    vbin[v] = bins(d);
    if (vbin[v] >= max_bins) return -1;
  }
  for (uint32_t v = 0; v < n; ++v) {
    uint32_t b = vbin[v];
    for (uint64_t x = rowptr[v]; x < rowptr[v + 1]; ++x) {
      for (uint64_t y = x + 1; y < rowptr[v + 1]; ++y) {
        uint32_t a = col[x], c = col[y];
        if (has_edge(keys, m, a, c)) {
          int cls = 1 + (vbin[a] == b) + (vbin[c] == b);
          P[b * 4 + cls] += 1;
          P[(uint64_t)max_bins * 4 + 3] += 1;
        } else {
          P[b * 4 + 0] += 1;
          P[(uint64_t)max_bins * 4 + 0] += 1;
        }
      }
    }
  }
  return 0;
}

// Exact triangle count by the forward algorithm (orient every edge from the
// endpoint earlier in (degree, id) order; count common forward neighbours).
// An enumeration independent of the wedge view, as in the related work of
// Sec. 1.2.
uint64_t orc_triangles_forward(const uint64_t* rowptr, const uint32_t* col, uint32_t n) {
  auto before = [&](uint32_t x, uint32_t y) {
    uint64_t dx = rowptr[x + 1] - rowptr[x], dy = rowptr[y + 1] - rowptr[y];
    return dx < dy || (dx == dy && x < y);
  };
  std::vector<std::vector<uint32_t>> fwd(n);
  for (uint32_t v = 0; v < n; ++v)
    for (uint64_t x = rowptr[v]; x < rowptr[v + 1]; ++x)
      if (before(v, col[x])) fwd[v].push_back(col[x]);
  for (auto& f : fwd) std::sort(f.begin(), f.end());
  uint64_t t = 0;
  for (uint32_t u = 0; u < n; ++u) {
    for (uint32_t w : fwd[u]) {
      const auto& A = fwd[u];
      const auto& B = fwd[w];
      size_t i = 0, j = 0;
      while (i < A.size() && j < B.size()) {
        if (A[i] < B[j]) ++i;
        else if (A[i] > B[j]) ++j;
        else { ++t; ++i; ++j; }
      }
    }
  }
  return t;
}

// ------------------------------------------------- control-variate pair table
// Bucket of a degree: floor(8 L(d)) with L Mitchell's log2,
// L(d) = e + (d - 2^e)/2^e, e = floor(log2 d): 8e + floor(8 (d - 2^e) / 2^e).
uint32_t orc_bucket(uint64_t d) {
  if (d == 0) return 0;
  uint32_t e = 63 - (uint32_t)__builtin_clzll(d);
  uint64_t p = (uint64_t)1 << e;
  return 8 * e + (uint32_t)(((d - p) * 8) / p);
}

// Census of every wedge by (centre bin, centre bucket, smaller endpoint
// bucket, larger endpoint bucket), by enumeration of all neighbour pairs of
// every centre (Sec. 2.1).  Entry for bin b, centre bucket k and bucket pair
// (i <= j) at ((b * 256 + k) * 256 + i) * 256 + j of out[max_bins*256^3]
// (caller zeroes; small graphs only).
int orc_pair_census(const uint64_t* rowptr, const uint32_t* col, uint32_t n, uint32_t tau,
                    uint64_t omega, uint32_t max_bins, uint64_t* out) {
  BinTable bins(tau, omega, max_bins);
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    if (d < 2) continue;
    uint32_t b = bins(d);
    if (b >= max_bins) return -1;
    uint32_t k = orc_bucket(d);
    for (uint64_t x = rowptr[v]; x < rowptr[v + 1]; ++x)
      for (uint64_t y = x + 1; y < rowptr[v + 1]; ++y) {
        uint32_t a = col[x], c = col[y];
        uint32_t ba = orc_bucket(rowptr[a + 1] - rowptr[a]);
        uint32_t bc = orc_bucket(rowptr[c + 1] - rowptr[c]);
        uint32_t i = ba < bc ? ba : bc, j = ba < bc ? bc : ba;
        out[(((uint64_t)b * 256 + k) * 256 + i) * 256 + j] += 1;
      }
  }
  return 0;
}

// ---------------------------------------------------------------- estimates
// Alg. phase4c summary and Eq. global_est, in double, in this order:
//   c_b = (q1+q2+q3)/k_b;  t_b = (p_b * (6q1+3q2+2q3)) / (6 k_b)
//   eps_b = sqrt(ln(2/delta) / (2 k_b))                      (Thm Hoeffding)
//   c = (sum_b p_b c_b) / p;  t = c p / 3
//   global stream: c_G = closed/k_G;  t_G = c_G p / 3
// out_bins[b*4 + {0,1,2,3}] = {c_b, t_b, eps_b, valid}; out_glob[0..5] =
// {c, t, c_G, t_G, eps_G, sum_b t_b}.
void orc_estimate(const uint64_t* p_b, const uint64_t* q, const uint64_t* k_per_bin,
                  uint32_t max_bins, uint64_t k_global, double delta, double* out_bins,
                  double* out_glob) {
  uint64_t p = 0;
  for (uint32_t b = 0; b < max_bins; ++b) p += p_b[b];
  double num = 0.0, tsum = 0.0;
  for (uint32_t b = 0; b < max_bins; ++b) {
    const uint64_t* qb = q + (uint64_t)b * 4;
    double c = 0.0, t = 0.0, e = 0.0, valid = 0.0;
    if (k_per_bin[b] > 0) {
      c = (double)(qb[1] + qb[2] + qb[3]) / (double)k_per_bin[b];
      uint64_t T6 = 6 * qb[1] + 3 * qb[2] + 2 * qb[3];
      t = ((double)p_b[b] * (double)T6) / (6.0 * (double)k_per_bin[b]);
      e = std::sqrt(std::log(2.0 / delta) / (2.0 * (double)k_per_bin[b]));
      valid = 1.0;
    }
    out_bins[b * 4 + 0] = c;
    out_bins[b * 4 + 1] = t;
    out_bins[b * 4 + 2] = e;
    out_bins[b * 4 + 3] = valid;
    num += (double)p_b[b] * c;
    tsum += t;
  }
  double cw = p > 0 ? num / (double)p : 0.0;
  out_glob[0] = cw;
  out_glob[1] = cw * (double)p / 3.0;
  const uint64_t* qg = q + (uint64_t)max_bins * 4;
  double cg = k_global > 0 ? (double)qg[3] / (double)k_global : 0.0;
  out_glob[2] = cg;
  out_glob[3] = cg * (double)p / 3.0;
  out_glob[4] = k_global > 0 ? std::sqrt(std::log(2.0 / delta) / (2.0 * (double)k_global)) : 0.0;
  out_glob[5] = tsum;
}

}  // extern "C"
