/* Seeded synthetic graph generators (input generation only).
 *
 * This module holds none of the wedge-sampling arithmetic: it only writes
 * raw undirected edge lists (with possible self-loops and duplicates, as a
 * generator produces them) that both the CPU oracle and the GPU path take as
 * input.  Shapes follow the paper's workloads (Sec. 5.1): Graph500-style
 * R-MAT / stochastic Kronecker graphs with generator matrix
 * [0.57 0.19; 0.19 0.05], heavy-tailed Chung-Lu graphs, and a community-
 * structured heavy-tailed graph built from dense Erdos-Renyi blocks plus
 * Chung-Lu edges (a BTER-like stand-in for the web crawls).
 *
 * Random numbers: a counter-based SplitMix64 mix (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) of
 * (seed, stream, index), so every edge can be generated independently and
 * the output does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t rnd(uint64_t seed, uint64_t stream, uint64_t i) {
  return mix64(mix64(seed * 0x9E3779B97F4A7C15ULL + stream * 0xD1B54A32D192ED03ULL + 1) +
               i * 0x9E3779B97F4A7C15ULL);
}

static inline double unit53(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Bijection of [0, 2^scale): xor key, odd multiply and xorshift, 4 rounds.
 * Used to relabel R-MAT vertices so hubs are not packed at low ids. */
static inline uint32_t relabel(uint32_t x, uint32_t scale, uint64_t seed) {
  uint64_t mask = (scale >= 32) ? 0xFFFFFFFFULL : ((1ULL << scale) - 1);
  uint64_t y = x;
  uint32_t sh = (scale + 1) / 2;
  if (sh == 0) sh = 1;
  for (int r = 0; r < 4; ++r) {
    y ^= rnd(seed, 2, (uint64_t)r) & mask;
    y = (y * (rnd(seed, 3, (uint64_t)r) | 1)) & mask;
    y ^= y >> sh;
  }
  return (uint32_t)(y & mask);
}

/* R-MAT: each edge descends `scale` levels of the 2x2 generator matrix
 * (a, b; c, d = 1-a-b-c), one 32-bit uniform per level.  Vertex ids are
 * relabelled by a seeded bijection when `permute` is set. */
void synth_rmat(uint32_t scale, uint64_t n_edges, double a, double b, double c, uint64_t seed,
                int permute, uint32_t* src, uint32_t* dst) {
  const uint64_t ta = (uint64_t)(a * 4294967296.0);
  const uint64_t tb = (uint64_t)((a + b) * 4294967296.0);
  const uint64_t tc = (uint64_t)((a + b + c) * 4294967296.0);
  const uint64_t words = (scale + 1) / 2;
#pragma omp parallel for schedule(static)
  for (int64_t ei = 0; ei < (int64_t)n_edges; ++ei) {
    uint64_t e = (uint64_t)ei;
    uint32_t u = 0, v = 0;
    uint64_t r = 0;
    for (uint32_t l = 0; l < scale; ++l) {
      if ((l & 1) == 0) r = rnd(seed, 1, e * words + l / 2);
      uint64_t x = (l & 1) ? (r >> 32) : (r & 0xFFFFFFFFULL);
      uint32_t qu = 0, qv = 0;
      if (x < ta) {
      } else if (x < tb) {
        qv = 1;
      } else if (x < tc) {
        qu = 1;
      } else {
        qu = 1; qv = 1;
      }
      u = (u << 1) | qu;
      v = (v << 1) | qv;
    }
    if (permute) {
      u = relabel(u, scale, seed);
      v = relabel(v, scale, seed);
    }
    src[e] = u;
    dst[e] = v;
  }
}

/* Discrete power law on [wmin, wmax] with P(w) ~ w^-gamma, by inverse CDF. */
static void power_law_weights(uint32_t n, double gamma, uint32_t wmin, uint32_t wmax,
                              uint64_t seed, uint64_t stream, uint32_t* w) {
  uint32_t K = wmax - wmin + 1;
  double* cdf = (double*)malloc(sizeof(double) * K);
  double acc = 0.0;
  for (uint32_t i = 0; i < K; ++i) {
    acc += pow((double)(wmin + i), -gamma);
    cdf[i] = acc;
  }
  for (uint32_t i = 0; i < K; ++i) cdf[i] /= acc;
  cdf[K - 1] = 1.0;
#pragma omp parallel for schedule(static)
  for (int64_t vi = 0; vi < (int64_t)n; ++vi) {
    double u = unit53(rnd(seed, stream, (uint64_t)vi));
    uint32_t lo = 0, hi = K - 1; /* first i with cdf[i] > u */
    while (lo < hi) {
      uint32_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    w[vi] = wmin + lo;
  }
  free(cdf);
}

/* Weighted vertex choice: the first v with cum[v] > x for x = floor(r total /
 * 2^64).  A guide table over equal slices of [0, total) narrows the binary
 * search to the vertices whose cumulative weight ends inside x's slice. */
typedef struct {
  const uint64_t* cum;
  uint32_t n;
  uint64_t total;
  uint64_t step;
  uint32_t* guide; /* [J + 1]: first v with cum[v] > j step (n - 1 past the end) */
} Picker;

static void picker_init(Picker* p, const uint64_t* cum, uint32_t n, uint64_t total) {
  uint64_t J = n / 2 + 1;
  if (J > (1u << 26)) J = 1u << 26;
  p->cum = cum;
  p->n = n;
  p->total = total;
  p->step = total / J + 1; /* J step > total */
  p->guide = (uint32_t*)malloc(sizeof(uint32_t) * (J + 1));
  uint32_t v = 0;
  for (uint64_t j = 0; j <= J; ++j) {
    const uint64_t t = j * p->step;
    while (v < n - 1 && cum[v] <= t) ++v;
    p->guide[j] = v;
  }
}

static inline uint32_t pick_weighted(const Picker* p, uint64_t r) {
  const uint64_t x = (uint64_t)(((u128)r * p->total) >> 64); /* in [0, total) */
  const uint64_t j = x / p->step;
  uint32_t lo = p->guide[j], hi = p->guide[j + 1];
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (p->cum[mid] > x) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* Chung-Lu ("fast" edge-draw form): expected degrees w_v from a discrete
 * power law; each of the M edges picks both endpoints with probability
 * proportional to w.  Self-loops and duplicates are left for the consumer
 * to remove.  weights_out (nullable) receives w. */
void synth_chung_lu(uint32_t n, double gamma, uint32_t wmin, uint32_t wmax, uint64_t M,
                    uint64_t seed, uint32_t* src, uint32_t* dst, uint32_t* weights_out) {
  uint32_t* w = weights_out ? weights_out : (uint32_t*)malloc(sizeof(uint32_t) * n);
  power_law_weights(n, gamma, wmin, wmax, seed, 10, w);
  uint64_t* cum = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t acc = 0;
  for (uint32_t v = 0; v < n; ++v) {
    acc += w[v];
    cum[v] = acc;
  }
  Picker pk;
  picker_init(&pk, cum, n, acc);
#pragma omp parallel for schedule(static)
  for (int64_t ei = 0; ei < (int64_t)M; ++ei) {
    src[ei] = pick_weighted(&pk, rnd(seed, 11, 2 * (uint64_t)ei));
    dst[ei] = pick_weighted(&pk, rnd(seed, 11, 2 * (uint64_t)ei + 1));
  }
  free(pk.guide);
  free(cum);
  if (!weights_out) free(w);
}

/* BTER-like community graph.  Target degrees from a discrete power law on
 * [dmin, dmax] (exponent gamma).  Vertices sorted by target degree are cut
 * greedily into blocks of d+1 consecutive vertices (d = target degree of the
 * block's first vertex); inside a block every pair is an edge with
 * probability rho_d = min(1, 1/ln d).  The block stops being formed when
 * fewer than d+1 vertices remain.  Each vertex's remaining expected degree
 * (target minus expected in-block degree) is filled by Chung-Lu edges.
 * Returns the number of edges written (<= cap); *needed receives the total
 * the generator wanted to write, so a caller can size `cap`. */
uint64_t synth_bter(uint32_t n, double gamma, uint32_t dmin, uint32_t dmax, uint64_t seed,
                    uint32_t* src, uint32_t* dst, uint64_t cap, uint64_t* needed) {
  uint32_t* d = (uint32_t*)malloc(sizeof(uint32_t) * n);
  power_law_weights(n, gamma, dmin, dmax, seed, 20, d);
  /* counting sort of vertex ids by target degree (ascending) */
  uint64_t K = (uint64_t)dmax + 2;
  uint64_t* cnt = (uint64_t*)calloc(K, sizeof(uint64_t));
  for (uint32_t v = 0; v < n; ++v) cnt[d[v] + 1]++;
  for (uint64_t i = 1; i < K; ++i) cnt[i] += cnt[i - 1];
  uint32_t* ord = (uint32_t*)malloc(sizeof(uint32_t) * n);
  for (uint32_t v = 0; v < n; ++v) ord[cnt[d[v]]++] = v;
  free(cnt);
  /* blocks */
  uint64_t nblk = 0;
  uint32_t* bstart = (uint32_t*)malloc(sizeof(uint32_t) * (n / 2 + 2));
  uint32_t* bsize = (uint32_t*)malloc(sizeof(uint32_t) * (n / 2 + 2));
  double* excess = (double*)malloc(sizeof(double) * n);
  for (uint32_t v = 0; v < n; ++v) excess[v] = d[v];
  uint64_t pos = 0;
  while (pos < n) {
    uint32_t dd = d[ord[pos]];
    uint64_t sz = (uint64_t)dd + 1;
    if (pos + sz > n) break;
    bstart[nblk] = (uint32_t)pos;
    bsize[nblk] = (uint32_t)sz;
    double rho = dd >= 3 ? fmin(1.0, 1.0 / log((double)dd)) : 1.0;
    for (uint64_t i = pos; i < pos + sz; ++i) {
      double e = excess[ord[i]] - rho * (double)dd;
      excess[ord[i]] = e > 0 ? e : 0;
    }
    ++nblk;
    pos += sz;
  }
  /* in-block edges: pair (i, j) of block B kept iff rnd < rho */
  uint64_t* boff = (uint64_t*)malloc(sizeof(uint64_t) * (nblk + 1));
  boff[0] = 0;
  for (uint64_t bI = 0; bI < nblk; ++bI) {
    uint64_t s = bsize[bI];
    boff[bI + 1] = boff[bI] + s * (s - 1) / 2;
  }
  /* Chung-Lu fill over the excess, total expected degree sum */
  uint64_t* cum = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t acc = 0;
  for (uint32_t v = 0; v < n; ++v) {
    acc += (uint64_t)llround(excess[v] * 16.0);
    cum[v] = acc;
  }
  uint64_t ncl = (uint64_t)((double)acc / 16.0 / 2.0);
  /* count in-block edges per block (parallel), then prefix, then write */
  uint64_t* bcount = (uint64_t*)calloc(nblk + 1, sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t bI = 0; bI < (int64_t)nblk; ++bI) {
    uint32_t dd = bsize[bI] - 1;
    double rho = dd >= 3 ? fmin(1.0, 1.0 / log((double)dd)) : 1.0;
    uint64_t thr = rho >= 1.0 ? ~0ULL : (uint64_t)(rho * 18446744073709551616.0);
    uint64_t c = 0;
    for (uint64_t pI = boff[bI]; pI < boff[bI + 1]; ++pI)
      if (rho >= 1.0 || rnd(seed, 21, pI) < thr) ++c;
    bcount[bI + 1] = c;
  }
  for (uint64_t bI = 0; bI < nblk; ++bI) bcount[bI + 1] += bcount[bI];
  uint64_t nblock_edges = bcount[nblk];
  uint64_t total = nblock_edges + ncl;
  if (needed) *needed = total;
  if (src && dst && total <= cap) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t bI = 0; bI < (int64_t)nblk; ++bI) {
      uint32_t s = bsize[bI];
      uint32_t dd = s - 1;
      double rho = dd >= 3 ? fmin(1.0, 1.0 / log((double)dd)) : 1.0;
      uint64_t thr = rho >= 1.0 ? ~0ULL : (uint64_t)(rho * 18446744073709551616.0);
      uint64_t out = bcount[bI];
      uint64_t pI = boff[bI];
      for (uint32_t i = 0; i < s; ++i)
        for (uint32_t j = i + 1; j < s; ++j, ++pI)
          if (rho >= 1.0 || rnd(seed, 21, pI) < thr) {
            src[out] = ord[bstart[bI] + i];
            dst[out] = ord[bstart[bI] + j];
            ++out;
          }
    }
    if (acc > 0) {
      Picker pk;
      picker_init(&pk, cum, n, acc);
#pragma omp parallel for schedule(static)
      for (int64_t ei = 0; ei < (int64_t)ncl; ++ei) {
        src[nblock_edges + ei] = pick_weighted(&pk, rnd(seed, 22, 2 * (uint64_t)ei));
        dst[nblock_edges + ei] = pick_weighted(&pk, rnd(seed, 22, 2 * (uint64_t)ei + 1));
      }
      free(pk.guide);
    }
  }
  free(d); free(ord); free(bstart); free(bsize); free(excess); free(boff); free(cum); free(bcount);
  return (src && dst && total <= cap) ? total : 0;
}

/* Batch recipe: scale and edge factor of graph g of a batch, drawn from the
 * batch seed: scale in [smin, smax], edge factor in [emin, emax]. */
void synth_batch_shape(uint64_t seed, uint32_t g, uint32_t smin, uint32_t smax, uint32_t emin,
                       uint32_t emax, uint32_t* scale, uint32_t* edgefactor) {
  uint64_t r0 = rnd(seed, 30, 2 * (uint64_t)g), r1 = rnd(seed, 30, 2 * (uint64_t)g + 1);
  *scale = smin + (uint32_t)(((u128)r0 * (smax - smin + 1)) >> 64);
  *edgefactor = emin + (uint32_t)(((u128)r1 * (emax - emin + 1)) >> 64);
}
