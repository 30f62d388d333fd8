/* wedge.h -- C ABI of libwedge: wedge sampling of triangle statistics on an
 * MI355X (gfx950).
 *
 * Method: Kolda, Pinar, Plantenga, Seshadhri, Task, "Counting Triangles in
 * Massive Graphs with MapReduce" (arXiv 1301.5887).  The calls follow the
 * paper's statement of the problem: an undirected edge list in no particular
 * order with no meaning given to self-loops or repeats (Sec. 4.1, Sec. 5.1),
 * degree bins set by (tau, omega) (Sec. 4.2), k samples per bin set by
 * (eps, delta) (Sec. 3.1), and per-bin and global clustering coefficients and
 * triangle counts as output (Alg. phase4c, Eq. global_est).
 *
 * Conventions for every call:
 *  - Pointers named d_* or documented "device" are device (HBM) pointers;
 *    pointers named h_* are host pointers.  The caller owns and allocates
 *    every buffer (sizes come from the *_workspace / *_bytes queries); the
 *    library allocates nothing.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Device work is
 *    enqueued asynchronously on it; no call synchronises except those whose
 *    description says so (wedge_index_status, the autotuners, calls that
 *    read a count back before sizing their next step, wedge_sample_stream).
 *  - Return value: WEDGE_OK (0) or a negative wedge_status.  Arguments are
 *    validated on the host before anything is enqueued; on error nothing is
 *    enqueued, outputs are untouched and wedge_last_error() returns a message
 *    (thread-local).  Conditions only the device can see (an edge id >= n,
 *    a degree whose bin is >= max_bins) are reported in device-side counters
 *    documented per call.
 *  - Vertex ids are uint32 (n < 2^32); edge offsets are uint64.
 */
#ifndef WEDGE_H
#define WEDGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WEDGE_OK = 0,
  WEDGE_EINVAL = -1,     /* null or misaligned pointer, inconsistent arguments */
  WEDGE_ERANGE = -2,     /* a size or parameter outside the supported range */
  WEDGE_EWORKSPACE = -3, /* workspace or output buffer smaller than required */
  WEDGE_EHIP = -4,       /* a HIP runtime call or kernel launch failed */
  WEDGE_ENOTSUP = -5,    /* no usable gfx950 device */
  WEDGE_EGRAPH = -6      /* the adjacency is not a sorted simple undirected graph
                            (only with WEDGE_VALIDATE=1; see wedge_validate_csr),
                            or a streamed edge list is not simple */
} wedge_status;

/* Message of the last failed call on this thread ("" if none). */
const char* wedge_last_error(void);

/* Version of this ABI (incremented on any incompatible change). */
int wedge_abi_version(void);

/* ------------------------------------------------------------------------
 * Degree binning, Sec. 4.2 (Eqs. binlodeg, binid), integer form.
 * BinLoDeg(b) = b for b <= tau, else tau + sum_{j<b-tau} omega^j (saturating
 * at 2^64-1); BinId(d) = max{ b : BinLoDeg(b) <= d } for d >= 1.  With
 * tau = omega = 2 the bins are {1},{2},{3,4},{5..8},...  Requires tau >= 1
 * and integer omega >= 2.  Host-only helpers.
 * ---------------------------------------------------------------------- */
uint64_t wedge_bin_lo_deg(uint32_t b, uint32_t tau, uint64_t omega);
uint32_t wedge_bin_id(uint64_t d, uint32_t tau, uint64_t omega);

/* Thm. Hoeffding: k = ceil(0.5 * eps^-2 * ln(2/delta)) samples give
 * |c_hat - c| < eps with probability >= 1 - delta.  Returns 0 unless
 * 0 < eps and 0 < delta < 1.  Host-only. */
uint64_t wedge_hoeffding_k(double eps, double delta);

/* ------------------------------------------------------------------------
 * wedge_build_csr -- degree per vertex and adjacency (Alg. phase1a and the
 * input convention of Sec. 4.1: undirected, self-loops and repeats ignored).
 *
 * In:  d_src[m_in], d_dst[m_in]  device uint32 edge endpoints, any order.
 * Out: d_rowptr[n+1]  device uint64; row v of the adjacency is
 *                     d_col[d_rowptr[v] .. d_rowptr[v+1]), so the degree is
 *                     d_rowptr[v+1] - d_rowptr[v].
 *      d_col[2*m_in]  device uint32 capacity; the first 2m entries hold every
 *                     neighbour of every vertex once, each row ascending.
 *      d_info[2]      device uint64: [0] = m, the number of distinct
 *                     undirected non-loop edges; [1] = number of input edges
 *                     rejected because an endpoint was >= n (they are
 *                     dropped; the caller decides whether that is an error).
 *                     [0] = 2^64 - 1 means a bounded wait between tiles (of
 *                     the sort or of the compaction) gave up and rowptr/col
 *                     are invalid (not expected: a tile only waits on tiles
 *                     that are already running).
 * Workspace: wedge_build_csr_workspace(m_in, n) bytes of device memory,
 * 256-byte aligned, contents ignored on entry.
 * Errors: EINVAL (null/misaligned pointer), ERANGE (n == 0, m_in >= 2^40),
 *         EWORKSPACE, EHIP.
 * ---------------------------------------------------------------------- */
size_t wedge_build_csr_workspace(uint64_t m_in, uint32_t n);
int wedge_build_csr(const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_in, uint32_t n,
                    uint64_t* d_rowptr, uint32_t* d_col, uint64_t* d_info, void* d_workspace,
                    size_t workspace_bytes, void* stream);

/* wedge_build_csr_noalloc -- wedge_build_csr with no workspace argument and
 * no device allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same inputs, outputs, results and device-side conditions as
 * wedge_build_csr for m_in <= 2^20 input edges; the workspace is a
 * file-scope device array of the library (36 MiB per GPU the library runs
 * on, held until the process ends), which the call clears where the build
 * needs zeros.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (on different streams or host threads) race and give
 * wrong results; serialise them.
 * Errors: EWORKSPACE (m_in > 2^20), ERANGE (n == 0), EINVAL (null or
 *         misaligned pointer), EHIP. */
int wedge_build_csr_noalloc(const uint32_t* d_src, const uint32_t* d_dst, uint64_t m_in,
                            uint32_t n, uint64_t* d_rowptr, uint32_t* d_col, uint64_t* d_info,
                            void* stream);

/* ------------------------------------------------------------------------
 * wedge_validate_csr -- device check that an adjacency has the form the path
 * assumes: the paper's input is an undirected graph without repeated edges
 * or self-loops (Sec. 4.1), so in sorted rows every row is strictly
 * ascending, no vertex is in its own row, and w is in row v exactly when v
 * is in row w.  wedge_build_csr always produces that form; callers that bring
 * their own rowptr/col can check it.
 * Out: d_counts[4] device uint64, overwritten: [0] entries not above their
 *      predecessor in the row (unsorted or repeated), [1] self-loops, [2]
 *      entries (v, w) without (w, v), [3] structural faults (rowptr[0] != 0,
 *      rowptr decreasing, rowptr[n] != 2m, an id >= n).  All zero = valid.
 * Asynchronous on the stream.  With the environment variable WEDGE_VALIDATE
 * set (not "0"), wedge_sample_close runs this check first (its d_q as the
 * counts), waits for it, and returns WEDGE_EGRAPH when a count is nonzero.
 * Errors: EINVAL, ERANGE (n == 0), EHIP.
 * ---------------------------------------------------------------------- */
int wedge_validate_csr(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                       uint64_t* d_counts, void* stream);

/* ------------------------------------------------------------------------
 * wedge_bin_counts -- wedges per vertex and per bin (Alg. phase1b, Sec. 2.1:
 * p_v = d_v (d_v - 1) / 2, degree-0 vertices ignored) and the sampling index
 * that draws a centre with probability p_v / p_b (Sec. 3.2).
 *
 * In:  d_rowptr[n+1] as produced by wedge_build_csr; m = d_info[0] (sizes
 *      the index; pass the same n, m, max_bins to wedge_sample_close).
 * Out: d_n_b[max_bins], d_p_b[max_bins]  device uint64: vertices and wedges
 *                     per bin (bins 0 and 1 never hold wedges).
 *      d_index        device blob of wedge_index_bytes(n, m, max_bins) bytes
 *                     (256-byte aligned): the centres ordered by
 *                     (degree, id), the table of distinct degrees with their
 *                     cumulative wedge counts, and per-bin ranges.  Opaque;
 *                     only wedge_sample_close and wedge_index_status read it.
 * Workspace: wedge_bin_counts_workspace(n) bytes.
 * Device-side condition: a degree whose bin is >= max_bins is counted in the
 * index's overflow counter (read it with wedge_index_status); those vertices
 * are left out of every bin.  overflow = 2^64 - 1 means the sort of the
 * centre order gave up waiting between tiles and the index is invalid (not
 * expected, as for wedge_build_csr).
 * Errors: EINVAL, ERANGE (tau == 0, omega < 2, max_bins == 0 or > 4096),
 *         EWORKSPACE, EHIP.
 * ---------------------------------------------------------------------- */
size_t wedge_index_bytes(uint32_t n, uint64_t m, uint32_t max_bins);
size_t wedge_bin_counts_workspace(uint32_t n);
int wedge_bin_counts(const uint64_t* d_rowptr, uint32_t n, uint64_t m, uint32_t tau,
                     uint64_t omega, uint32_t max_bins, uint64_t* d_n_b, uint64_t* d_p_b,
                     void* d_index, size_t index_bytes, void* d_workspace,
                     size_t workspace_bytes, void* stream);

/* Synchronises `stream`, then reads the index header: number of distinct
 * degrees, vertices whose bin was >= max_bins, samples requested from a bin
 * without wedges by wedge_sample_close (skipped), and sampler workgroups that
 * found the index built for a different n, m or max_bins (skipped).  Any
 * out-pointer may be NULL. */
int wedge_index_status(const void* d_index, uint32_t* h_num_classes, uint64_t* h_overflow,
                       uint64_t* h_empty_bin_samples, uint64_t* h_mismatch, void* stream);

/* ------------------------------------------------------------------------
 * wedge_sample_close -- uniform wedge sampling per bin and exact closure
 * tests (Thms. cd-est and td-est; Alg. phase2c Sampling; Alg. phase3b;
 * Alg. phase4c classes).
 *
 * For every bin b < max_bins with h_k[b] > 0, samples s = 0..h_k[b]-1 are
 * drawn from Philox4x64-10 with key (seed, 1) and counter
 * (s, b, graph_id, r), r = retry round of the uniform-below draw:
 *   w = U(word 0, p_b) picks the centre v (centres of the bin in
 *       (degree, id) order, each taking p_v consecutive values of w);
 *   o = U(word 1, d(d-1)) picks the ordered neighbour pair
 *       i = o / (d-1), j = r + [r >= i] with r = o mod (d-1), neighbours
 *       numbered in ascending id order;
 *   the wedge (a, v, c) is closed iff {a, c} is an edge;
 *   class = 0 if open, else 1 + [BinId(d_a) = b] + [BinId(d_c) = b].
 * U(x, N) is Lemire's nearly-divisionless uniform integer on [0, N): when
 * the low product word falls below 2^64 mod N the draw moves to the same
 * word of retry round r+1.
 * A global stream of k_global samples draws from all wedges (counter word 1
 * = 0xFFFFFFFF); its closed wedges have class 3, open ones class 0.
 *
 * In:  d_rowptr, d_col of the graph, its n and m, and d_index built by
 *      wedge_bin_counts with the same n, m and max_bins; h_k[max_bins] host
 *      sample counts (0 for bins without wedges).
 * Out: d_q[(max_bins+1)*4]  device uint64, overwritten: d_q[4b + c] = number
 *                     of samples of bin b in class c; row max_bins is the
 *                     global stream.
 *      d_probe_loads  nullable device uint64[1], overwritten: total number of
 *                     adjacency words read by the closure searches.
 *      d_dump         nullable device wedge_sample_rec[(max_bins+1) *
 *                     dump_per_bin]: record s of row r at r*dump_per_bin + s
 *                     for s < dump_per_bin; other records untouched.
 * Samples requested from a bin whose p_b is 0 are skipped and counted in the
 * index header (wedge_index_status).
 * Errors: EINVAL, ERANGE (a k above 2^48, max_bins mismatch), EHIP.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t v;   /* centre */
  uint32_t a;   /* endpoint N(v)[i] */
  uint32_t c;   /* endpoint N(v)[j] */
  uint32_t cls; /* 0 open, 1..3 closed with cls vertices in the bin */
} wedge_sample_rec;

int wedge_sample_close(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                       const void* d_index, uint32_t max_bins, const uint64_t* h_k,
                       uint64_t k_global, uint64_t seed, uint32_t graph_id, uint64_t* d_q,
                       uint64_t* d_probe_loads, wedge_sample_rec* d_dump, uint64_t dump_per_bin,
                       void* stream);

/* Same computation with explicit launch shape: `lanes_in_flight` samples per
 * lane carried through the gather chain together (1, 2, 4 or 8) and
 * `samples_per_tile` samples per workgroup (rounded up to a multiple of
 * 256 * lanes_in_flight).  Results are identical for every shape; only the
 * speed differs.  Used by the autotuner. */
int wedge_sample_close_tuned(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                             uint64_t m, const void* d_index, uint32_t max_bins,
                             const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                             uint32_t graph_id, uint64_t* d_q, uint64_t* d_probe_loads,
                             wedge_sample_rec* d_dump, uint64_t dump_per_bin,
                             int lanes_in_flight, uint64_t samples_per_tile, void* stream);

/* ------------------------------------------------------------------------
 * Closure by an edge table (Alg. phase3b matches a wedge's endpoint pair
 * against the edge set by key; here the match is a lookup).  The table holds
 * every edge once as the key min << 32 | max in 2^bits slots of 8 bytes
 * (linear probing, a Fibonacci hash of the key; empty slot = all bits set),
 * with 2^bits >= 2m so at most half the slots are used.
 *
 * wedge_edge_hash_bits(m): the least bits >= 4 with 2^bits >= 2m.
 * wedge_edge_hash_build: clears d_table (device uint64[2^bits], caller-owned)
 *   and inserts the edge {v, w}, v < w, of every adjacency entry; d_full
 *   (device uint64[1], overwritten) counts keys that found no empty slot
 *   (not expected at that load).  Asynchronous.
 *   Errors: EINVAL, ERANGE (n == 0, bits outside [4, 40] or 2^bits < 2m), EHIP.
 * wedge_sample_close_hashed: wedge_sample_close (same samples, same counts,
 *   same dump) with the closure test a lookup in the table built from the
 *   same rowptr/col; d_probe_loads counts table slots read instead of
 *   adjacency words.  Errors: as wedge_sample_close, plus EINVAL (table) and
 *   ERANGE (bits).
 * ---------------------------------------------------------------------- */
uint32_t wedge_edge_hash_bits(uint64_t m);
int wedge_edge_hash_build(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                          uint64_t* d_table, uint32_t bits, uint64_t* d_full, void* stream);
int wedge_sample_close_hashed(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                              uint64_t m, const void* d_index, uint32_t max_bins,
                              const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                              uint32_t graph_id, uint64_t* d_q, uint64_t* d_probe_loads,
                              wedge_sample_rec* d_dump, uint64_t dump_per_bin,
                              const uint64_t* d_table, uint32_t bits, void* stream);

/* ------------------------------------------------------------------------
 * wedge_estimate -- Alg. phase4c summary and Eq. global_est, host FP64, in
 * this order (no FMA contraction):
 *   c_b = (q1+q2+q3) / k_b;   t_b = (p_b * (6 q1 + 3 q2 + 2 q3)) / (6 k_b)
 *   eps_b = sqrt(ln(2/delta) / (2 k_b))
 *   c = (sum over b ascending of p_b c_b) / p,  t = c p / 3,  p = sum_b p_b
 *   global stream: c_G = q_G3 / k_G,  t_G = c_G p / 3
 * Bins with k_b = 0 get c = t = eps = 0 and valid = 0.
 * In: h_n_b, h_p_b, h_k [max_bins]; h_q[(max_bins+1)*4] as from
 *     wedge_sample_close.  Out: h_bins[max_bins], *h_global.
 * Errors: EINVAL (null pointer, delta outside (0,1)).
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t bin;
  uint32_t valid;    /* 1 if the bin was sampled */
  uint64_t lo_deg;   /* BinLoDeg(bin) */
  uint64_t n_b, p_b, k_b;
  uint64_t q[4];
  double c;          /* estimated closed fraction of the bin's wedges */
  double t;          /* estimated triangles with a vertex in the bin */
  double eps;        /* Hoeffding half-width of c at confidence 1 - delta */
} wedge_bin_estimate;

typedef struct {
  uint64_t p;        /* total wedges */
  uint64_t k_global;
  uint64_t q_global[4];
  double c;          /* sum_b (p_b/p) c_b */
  double t;          /* c p / 3 */
  double c_global;   /* global stream */
  double t_global;
  double eps_global;
  double t_bins_sum; /* sum_b t_b */
} wedge_global_estimate;

int wedge_estimate(const uint64_t* h_n_b, const uint64_t* h_p_b, const uint64_t* h_q,
                   const uint64_t* h_k, uint32_t max_bins, uint32_t tau, uint64_t omega,
                   uint64_t k_global, double delta, wedge_bin_estimate* h_bins,
                   wedge_global_estimate* h_global);


/* ------------------------------------------------------------------------
 * Batched form: many graphs of uneven size and all their degree bins, with
 * no host round trip between the steps (so the whole pipeline can be
 * captured into a HIP graph), one persistent sampler grid for every
 * (graph, bin) of the batch, and launch shapes chosen by an autotuner.
 *
 * Graph g owns input edges [edge_off[g], edge_off[g+1]) of d_src/d_dst with
 * ids local to the graph (0 <= id < n_g, others rejected), and the global
 * vertex ids [vert_off[g], vert_off[g+1]) with n_g = vert_off[g+1] -
 * vert_off[g] >= 1.  Every graph is sampled as by wedge_sample_close with
 * graph_id = g: bins with wedges get k_per_bin samples, the graph's global
 * stream k_global (0 when the graph has no wedges).  Sampled vertex ids are
 * global; the class counts of graph g equal those of the single-graph path
 * on graph g alone, bit for bit.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t num_graphs;     /* G >= 1 */
  uint32_t max_bins;       /* bins per graph, 1..4096 */
  uint32_t tau;            /* >= 1 */
  uint32_t max_n;          /* largest n_g; must be <= 2^(32 - bits(G-1)) */
  uint64_t omega;          /* integer >= 2 */
  uint64_t k_per_bin;      /* samples per bin with wedges, <= 2^48 */
  uint64_t k_global;       /* samples of each graph's global stream, <= 2^48 */
  uint64_t seed;           /* Philox key word 0 */
  uint64_t total_edges;    /* sum of the graphs' input edges, < 2^40 */
  uint64_t total_vertices; /* sum of n_g, < 2^32 */
} wedge_batch_desc;

/* Launch shape of the sampler: samples carried together per lane (1, 2, 4
 * or 8), samples per tile (rounded up to a multiple of 256 * lanes) and
 * workgroups of the persistent grid (0 = 2048).  Every shape gives the same
 * counts. */
typedef struct {
  int lanes_in_flight;
  uint32_t samples_per_tile;
  uint32_t workgroups;
} wedge_launch_shape;

/* Device workspace for a batch (0 if the descriptor is invalid).  It holds
 * the block-diagonal CSR, the index, the task table and scratch, and keeps
 * them between wedge_batch_prepare and wedge_batch_sample. */
size_t wedge_batch_workspace_bytes(const wedge_batch_desc* d);

/* Degrees, adjacency, bins and index of every graph (Alg. phase1a/1b).
 * In: d_src, d_dst [total_edges]; d_edge_off [G+1] (uint64, device);
 * d_vert_off [G+1] (uint32, device).  Out: d_n_b, d_p_b [G * max_bins]. */
int wedge_batch_prepare(const wedge_batch_desc* d, const uint32_t* d_src, const uint32_t* d_dst,
                        const uint64_t* d_edge_off, const uint32_t* d_vert_off, uint64_t* d_n_b,
                        uint64_t* d_p_b, void* d_workspace, size_t workspace_bytes, void* stream);

/* Samples and closure tests of every (graph, bin) of a prepared batch in one
 * persistent launch (Thms. cd-est/td-est, Alg. phase3b, Alg. phase4c), then
 * per-graph FP64 estimates on the device.  shape may be NULL (default).
 * Out: d_q [G * (max_bins+1) * 4] (row g*(max_bins+1) + b; row
 * g*(max_bins+1) + max_bins = global stream of g); d_probe_loads (nullable)
 * as in wedge_sample_close; d_est_glob (nullable) [G * 6] = c, t, c_G, t_G,
 * eps_G, sum_b t_b; d_est_bins (nullable) [G * max_bins * 3] = c_b, t_b,
 * eps_b, in the order and formulas of wedge_estimate. */
int wedge_batch_sample(const wedge_batch_desc* d, const wedge_launch_shape* shape, double delta,
                       uint64_t* d_q, uint64_t* d_probe_loads, double* d_est_glob,
                       double* d_est_bins, void* d_workspace, size_t workspace_bytes,
                       void* stream);

/* wedge_batch_prepare followed by wedge_batch_sample. */
int wedge_batch_run(const wedge_batch_desc* d, const uint32_t* d_src, const uint32_t* d_dst,
                    const uint64_t* d_edge_off, const uint32_t* d_vert_off,
                    const wedge_launch_shape* shape, double delta, uint64_t* d_n_b,
                    uint64_t* d_p_b, uint64_t* d_q, double* d_est_glob, double* d_est_bins,
                    void* d_workspace, size_t workspace_bytes, void* stream);

/* Captures wedge_batch_run with these arguments into a HIP graph (on a
 * private stream) and instantiates it; *h_graph receives an opaque handle.
 * Replays read and write the same buffers. */
int wedge_batch_graph_create(const wedge_batch_desc* d, const uint32_t* d_src,
                             const uint32_t* d_dst, const uint64_t* d_edge_off,
                             const uint32_t* d_vert_off, const wedge_launch_shape* shape,
                             double delta, uint64_t* d_n_b, uint64_t* d_p_b, uint64_t* d_q,
                             double* d_est_glob, double* d_est_bins, void* d_workspace,
                             size_t workspace_bytes, void** h_graph);
int wedge_batch_graph_launch(void* h_graph, void* stream);
int wedge_batch_graph_destroy(void* h_graph);

/* Autotuner of the batch sampler: runs every candidate shape `reps` times
 * on a prepared batch (synchronising), keeps the median time in h_ms[c],
 * checks that every candidate's counts equal candidate 0's (else EINVAL),
 * and sets *h_best to the fastest.  d_q_ref, d_q_try: [G*(max_bins+1)*4]. */
int wedge_batch_autotune(const wedge_batch_desc* d, const wedge_launch_shape* cands, int ncand,
                         int reps, uint64_t* d_q_ref, uint64_t* d_q_try, void* d_workspace,
                         size_t workspace_bytes, float* h_ms, int* h_best, void* stream);

/* Autotuner of the plain sampler: times wedge_sample_close on this graph and
 * index (with h_k, k_global and seed as given) under each candidate shape
 * (lanes_in_flight, samples_per_tile; workgroups unused by this launch form),
 * reps times each, h_ms[c] = the median ms; checks that every candidate's
 * class counts equal the first one's (d_q_ref, d_q_try: device uint64
 * [(max_bins+1)*4] scratch); *h_best = the fastest.  The pick is remembered
 * for (current device, n, m, max_bins) in a process-wide table:
 * wedge_sample_close then launches graphs of that size with it (results are
 * identical for every shape).  Synchronises the stream.
 * Errors: EINVAL (bad arguments, counts that differ), those of
 * wedge_sample_close, EHIP. */
int wedge_sample_close_autotune(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                                uint64_t m, const void* d_index, uint32_t max_bins,
                                const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                                const wedge_launch_shape* cands, int ncand, int reps,
                                uint64_t* d_q_ref, uint64_t* d_q_try, float* h_ms, int* h_best,
                                void* stream);
/* The shape wedge_sample_close uses for a graph of (n, m, max_bins) on the
 * current device: the autotuner's pick, or the default (1, 256). */
int wedge_sample_close_shape(uint32_t n, uint64_t m, uint32_t max_bins,
                             wedge_launch_shape* h_shape);

/* ------------------------------------------------------------------------
 * Learned control variate.  A small network g(x) in (0, 1) predicts the
 * closure probability of a sampled wedge from its degrees; the estimate of a
 * bin's closed fraction c_b (Thm. cd-est) becomes
 *     c_CV = mean_EVAL(X - beta g) + beta mean_AUX(g),
 * with beta fixed before the EVAL and AUX draws, which are independent of
 * each other and of the training draws (distinct Philox key domains).  So
 * c_CV is unbiased for any network, every closure test stays exact, and
 * beta = 0 is plain wedge sampling.  mean_AUX(g) may be replaced by the
 * exact mean of g over the bin's wedges (wedge_cv_census below).
 *
 * Network: x = (K(d_v), K(min(d_a,d_c)), K(max(d_a,d_c))) / 256 and bin / 32,
 * K(d) = floor(8 L(d)) with L(d) = e + (d - 2^e)/2^e, e = floor(log2 d)
 * (Mitchell's log2) -- the log-degree in steps of 1/8, exact in BF16;
 * h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2), g = sigmoid(W3 h2 + b3),
 * 4 -> 64 -> 64 -> 1, GELU(a) = a/2 (1 + erf(a/sqrt 2)).  Weights are kept
 * in FP32 (master) and BF16 (used by the matrix-core products); products
 * accumulate in FP32.  Loss: binary cross-entropy of g against the exact
 * closure label, averaged over the batch; update: Adam (Kingma & Ba).
 * Parameter vector order (4545 floats): W1[64][4], b1[64], W2[64][64],
 * b2[64], W3[64], b3.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t dv;      /* centre degree */
  uint32_t dlo;     /* smaller endpoint degree */
  uint32_t dhi;     /* larger endpoint degree */
  uint16_t bin;     /* BinId(dv) */
  uint8_t closed;   /* exact closure label (0 when the search was skipped) */
  uint8_t cls;      /* class as in wedge_sample_close */
} wedge_feature_rec;

/* Philox key domains of the streams (key word 1). */
enum { WEDGE_DOMAIN_SAMPLE = 1, WEDGE_DOMAIN_TRAIN = 2, WEDGE_DOMAIN_AUX = 3,
       WEDGE_DOMAIN_EVAL = 4, WEDGE_DOMAIN_CENTRE = 6, WEDGE_DOMAIN_ALLOC = 7 };

/* The sampler of wedge_sample_close with key (seed, domain), samples
 * s = s_begin[r] .. s_begin[r] + h_k[r] - 1 of every row r (bins r < max_bins
 * and the global stream r = max_bins; h_k and h_s_begin have max_bins + 1
 * entries, h_s_begin nullable = all zero).  Rows with h_k[r] > 0, taken in
 * increasing r, fill record rows j = 0, 1, ...: the record of sample s of the
 * j-th such row goes to d_out[j * out_stride + (s - s_begin[r])].
 * closure = 0 skips the closure search (records get closed = cls = 0).
 * d_q (nullable) receives the class counts of these samples as in
 * wedge_sample_close.  Requires h_k[r] <= out_stride. */
int wedge_sample_features(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                          uint64_t m, const void* d_index, uint32_t max_bins, uint32_t tau,
                          uint64_t omega, const uint64_t* h_k, const uint64_t* h_s_begin,
                          uint64_t seed,
                          uint32_t domain, uint32_t graph_id, int closure,
                          wedge_feature_rec* d_out, uint64_t out_stride, uint64_t* d_q,
                          void* stream);

/* Network state on the device: FP32 master weights, BF16 copy, Adam
 * moments.  wedge_mlp_state_bytes() bytes, 256-byte aligned. */
size_t wedge_mlp_state_bytes(void);
/* Loads 4545 FP32 parameters (device pointer) into the state, makes the BF16
 * copy and clears the Adam moments. */
int wedge_mlp_set(void* d_state, const float* d_params, void* stream);
/* Copies the FP32 master parameters out (device pointer, 4545 floats). */
int wedge_mlp_get(const void* d_state, float* d_params, void* stream);
/* Fan-in-scaled uniform initialisation from Philox (key (seed, 5)). */
int wedge_mlp_init(void* d_state, uint64_t seed, void* stream);
/* g for n records (device FP32 out). */
int wedge_mlp_forward(const void* d_state, const wedge_feature_rec* d_x, uint64_t n, float* d_g,
                      void* stream);
/* Gradient (4545 FP32, device) and mean loss (1 FP32, device, nullable) of
 * the BCE loss (labels = closed) over the minibatch made of records
 * j0 .. j0 + per_row - 1 of each of the `rows` rows of d_x[rows][stride]
 * (n = rows * per_row records, so a minibatch can hold every bin).
 * Workspace: wedge_mlp_grad_workspace(n) bytes. */
size_t wedge_mlp_grad_workspace(uint64_t n);
int wedge_mlp_grad(const void* d_state, const wedge_feature_rec* d_x, uint32_t rows,
                   uint64_t stride, uint64_t j0, uint64_t per_row, float* d_grad, float* d_loss,
                   void* d_workspace, size_t workspace_bytes, void* stream);
/* One Adam step (t >= 1) of the master weights with gradient d_grad; the
 * BF16 copy is refreshed. */
int wedge_mlp_adam(void* d_state, const float* d_grad, uint32_t t, float lr, float beta1,
                   float beta2, float eps, void* stream);
/* Minibatch training as one sequence of device work: for each of `epochs`
 * passes over columns 0 .. n_fit - 1 of the `rows` rows of d_x[rows][stride]
 * (n_fit a multiple of per_row_batch, n_fit <= stride), minibatches of
 * per_row_batch consecutive columns of every row, each a wedge_mlp_grad
 * followed by a wedge_mlp_adam at steps t0 + 1, t0 + 2, ...  The loss of the
 * last minibatch goes to d_loss (device FP32, nullable).  Workspace:
 * wedge_mlp_train_workspace(rows, per_row_batch) bytes. */
size_t wedge_mlp_train_workspace(uint32_t rows, uint64_t per_row_batch);
int wedge_mlp_train(void* d_state, const wedge_feature_rec* d_x, uint32_t rows, uint64_t stride,
                    uint64_t n_fit, uint64_t per_row_batch, uint32_t epochs, uint32_t t0,
                    float lr, float beta1, float beta2, float eps, float* d_loss,
                    void* d_workspace, size_t workspace_bytes, void* stream);

/* Moments of the control variate over records d_x (rows x stride, the first
 * n_per_row of each row used, or the first h_counts[r] of row r when the host
 * array h_counts is given) with network outputs d_g (same layout), added
 * into d_mom[rows][5] (int64, caller zeroes); d_x may be null (X = 0, for
 * values without a closure label such as centre means):
 *   [0] count, [1] sum X, [2] round(2^32 sum g), [3] round(2^32 sum g^2),
 *   [4] round(2^32 sum X g)
 * with every term rounded to 2^-32 before summing, so sums are exact and
 * independent of order.  X = closed. */
int wedge_cv_moments(const wedge_feature_rec* d_x, const float* d_g, uint32_t rows,
                     uint64_t stride, uint64_t n_per_row, const uint64_t* h_counts,
                     int64_t* d_mom, void* stream);

/* Census of the wedges of every bin by (bin, centre bucket, endpoint bucket
 * pair), buckets K(d) = floor(8 L(d)) as in the network's features.  With
 * it the mean of the network over all wedges of bin b is the finite sum
 *   mu_b = (1/p_b) sum_keys sum_{i<=j} census[key][i,j] g(key, i, j),
 * which makes the control variate's mean exact (no auxiliary draws).
 * d_census: wedge_cv_census_bytes(n, m, max_bins) bytes, 256-byte aligned;
 * keys are the (bin, centre bucket) pairs degrees >= 2 can take, numbered in
 * increasing degree order; the count of key `key` and bucket pair
 * (i <= j < 256) is entry j (j + 1) / 2 + i of its row of 32896 uint64.  The
 * key list and the table sit at offsets that depend on max_bins only; the
 * rest of the buffer is per-graph scratch (a bucket byte per vertex and the
 * total degree before each degree class).
 * In: the graph and index as for wedge_sample_close. */
size_t wedge_cv_census_bytes(uint32_t n, uint64_t m, uint32_t max_bins);
int wedge_cv_census(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                    const void* d_index, uint32_t max_bins, uint32_t tau, uint64_t omega,
                    void* d_census, size_t census_bytes, void* stream);
/* Synchronises and reads the key list: *h_nkeys, and (nullable)
 * h_key_bin[], h_key_bucket[] (room for 256 + max_bins + 1 entries). */
int wedge_cv_census_keys(const void* d_census, uint32_t max_bins, uint32_t* h_nkeys,
                         uint32_t* h_key_bin, uint32_t* h_key_bucket, void* stream);
/* For every key: d_key_sum[key] = sum over its bucket pairs of
 * census * g (FP64, fixed summation order) and d_key_count[key] = its wedge
 * count (sums to p_b over the keys of bin b).  Reads the key count from the
 * device first (synchronises the stream).  Workspace:
 * wedge_cv_exact_mean_workspace(max_bins) bytes. */
size_t wedge_cv_exact_mean_workspace(uint32_t max_bins);
int wedge_cv_exact_mean(const void* d_state, const void* d_census, uint32_t max_bins,
                        double* d_key_sum, uint64_t* d_key_count, void* d_workspace,
                        size_t workspace_bytes, void* stream);

/* Key list only (no census counts): fills the (bin, bucket) keys of a buffer
 * of wedge_cv_census_bytes(n, m, max_bins) bytes, as wedge_cv_census does. */
int wedge_cv_keys(void* d_census, uint32_t max_bins, uint32_t tau, uint64_t omega, void* stream);
/* The network's g for every present key and every bucket pair (i <= j):
 * d_gtable[key * 32896 + j (j + 1) / 2 + i] (FP32, room for 256 + max_bins + 1
 * keys).  Reads the key count from the device first (synchronises the
 * stream).  Workspace: wedge_cv_gtable_workspace(max_bins) bytes. */
size_t wedge_cv_gtable_workspace(uint32_t max_bins);
int wedge_cv_gtable(const void* d_state, const void* d_census, uint32_t max_bins, float* d_gtable,
                    void* d_workspace, size_t workspace_bytes, void* stream);
/* Centre draws for the control variate's mean: draw s of row r (s =
 * s_begin[r] .. s_begin[r] + h_k[r] - 1, key (seed, domain)) picks a centre v
 * with probability p_v / p_r exactly as the sampler picks a wedge's centre
 * (Sec. 3.2), and d_out gets the mean of g over all C(d_v, 2) wedges at v,
 *   gbar(v) = (1 / C(d_v, 2)) sum over neighbour pairs of g(key(v), K(d_lo), K(d_hi)),
 * from the table of wedge_cv_gtable; E[gbar(v)] is the mean of g over the
 * row's wedges.  Rows with h_k[r] > 0, in increasing r, fill output rows
 * j = 0, 1, ...: draw s of the j-th such row goes to d_out[j * out_stride +
 * (s - s_begin[r])], and its centre id to d_vout (nullable) at the same place.
 * d_census holds the key list (wedge_cv_keys or wedge_cv_census).  Workspace:
 * wedge_cv_centre_means_workspace(sum of h_k) bytes. */
size_t wedge_cv_centre_means_workspace(uint64_t total_draws);
int wedge_cv_centre_means(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                          const void* d_index, uint32_t max_bins, uint32_t tau, uint64_t omega,
                          const uint64_t* h_k, const uint64_t* h_s_begin, uint64_t seed,
                          uint32_t domain, uint32_t graph_id, const void* d_census,
                          const float* d_gtable, float* d_out, uint64_t out_stride,
                          uint32_t* d_vout, void* d_workspace, size_t workspace_bytes,
                          void* stream);

/* ------------------------------------------------------------------------
 * wedge_sample_alloc -- the paper's own sample allocation (Alg. phase2a)
 * followed by the Sampling procedure of Alg. phase2c, as an alternative to
 * the i.i.d. draws of wedge_sample_close.
 *
 * For every row r (bin r < max_bins with h_k[r] > 0, and the global stream
 * r = max_bins when k_global > 0) each vertex v of the row with d >= 2 gets
 * q_v samples: q* = C(d,2) k_r / p_r rounded down, plus one with probability
 * equal to its fractional part exactly (E[q_v] = q*; the rounding draw of v
 * is uniform on [0, p_r) from word 2 of Philox blocks (v, row word, 0, retry)
 * under key (seed, WEDGE_DOMAIN_ALLOC) and rounds up iff it is below
 * (C(d,2) k_r) mod p_r).  The row's samples are numbered s = 0 .. Q_r - 1
 * through its vertices in the centre order (degree, id); sample s at v takes
 * the ordered neighbour pair of wedge_sample_close from word 1 of blocks
 * (s, row word, 0, retry), is closure-tested and classified as there.
 * Out: d_q[(max_bins+1)*4] class counts (overwritten); h_totals[max_bins+1]
 *      (host) the realised totals Q_r, the denominators of the estimates
 *      (pass them to wedge_estimate as the per-row sample counts);
 *      d_dump (nullable) as in wedge_sample_close.
 * Reads the totals back, so it synchronises the stream.  A row whose p_r is
 * 0 draws nothing.  Workspace: wedge_sample_alloc_workspace(n, max_bins).
 * Errors: as wedge_sample_close, plus EWORKSPACE.
 * ---------------------------------------------------------------------- */
size_t wedge_sample_alloc_workspace(uint32_t n, uint32_t max_bins);
int wedge_sample_alloc(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                       const void* d_index, uint32_t max_bins, const uint64_t* h_k,
                       uint64_t k_global, uint64_t seed, uint64_t* d_q, uint64_t* h_totals,
                       wedge_sample_rec* d_dump, uint64_t dump_per_bin, void* d_workspace,
                       size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * wedge_closure_join -- closure tests by a join against an unsorted edge
 * list streamed from host memory (the pattern of Alg. phase3b: the wedges'
 * endpoint pairs meet the edges by key, either orientation), for edge lists
 * that are not (or cannot be) held as a sorted adjacency in HBM.
 *
 * In:  d_a[k], d_c[k]  device uint32 endpoints of k wedges (a != c).
 *      h_src[m_in], h_dst[m_in]  host uint32 edge list, any order, repeats
 *                     and self-loops allowed; pinned memory lets the copies
 *                     overlap the probes; it must stay valid until the work
 *                     on `stream` has finished.
 *      chunk_edges    edges per copy (0: 2^24).
 * Out: d_closed[k]    device uint8: 1 iff {a_i, c_i} is an edge.
 * The pairs go into an open-addressing table (SplitMix64 hash, at most half
 * full); chunks of the edge list are copied on a second stream of the same
 * device (created on first use, default priority) into two alternating
 * buffers while the caller's stream probes the previous chunk.
 * Workspace: wedge_closure_join_workspace(k, chunk_edges) bytes.
 * Errors: EINVAL, ERANGE (k >= 2^40), EWORKSPACE, EHIP.
 * ---------------------------------------------------------------------- */
size_t wedge_closure_join_workspace(uint64_t k, uint64_t chunk_edges);
int wedge_closure_join(const uint32_t* d_a, const uint32_t* d_c, uint64_t k,
                       const uint32_t* h_src, const uint32_t* h_dst, uint64_t m_in,
                       uint64_t chunk_edges, uint8_t* d_closed, void* d_workspace,
                       size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * wedge_sample_stream -- wedge_bin_counts + wedge_sample_close on an edge
 * list held in host memory, with no adjacency on the device (the paper's
 * setting: every phase is a pass over the edge list, Alg. phase1a to
 * phase4c).  The edge list streams in chunks of chunk_edges (0: 2^24),
 * copies on a second stream overlapping the kernels:
 *   a degree pass (Alg. phase1a: a count per endpoint), then the bins and
 *   the sampling index (Alg. phase1b); the draws of wedge_sample_close (same
 *   Philox stream, centres and neighbour ranks i, j) without reading an
 *   adjacency; gather passes that collect and sort the edges of the drawn
 *   centres, a vertex range of at most gather_cap edge ends at a time, which
 *   turns (i, j) into the endpoints (Alg. phase2c: a centre sees all its
 *   edges); a closure join (Alg. phase3b, as wedge_closure_join); the
 *   classes of Alg. phase4c from the streamed degrees.
 * The input must be simple (no repeated edge, in either orientation; Sec.
 * 4.1 states the input that way): a degree is then a count.  Self-loops are
 * skipped; edges with an id >= n are skipped and counted in h_info[1].  For
 * such a list the bins, counts and records equal those of wedge_build_csr +
 * wedge_bin_counts + wedge_sample_close on the same list.
 *
 * In:  h_src[m_in], h_dst[m_in]  host uint32 edge list (pinned memory lets
 *                     the copies overlap); read in 2 + (gather rounds)
 *                     passes; must not change during the call.
 *      n, tau, omega, max_bins as wedge_bin_counts; h_k[max_bins],
 *      k_global, seed as wedge_sample_close (graph_id 0); a bin whose p_b
 *      turns out 0 gets no samples.
 *      gather_cap     largest number of edge ends one gather round holds
 *                     (its sort buffers: 16 bytes per end); it must be at
 *                     least the largest degree of a drawn centre.
 * Out: d_n_b[max_bins], d_p_b[max_bins] as wedge_bin_counts;
 *      d_q[(max_bins+1)*4] and d_dump (nullable, dump_per_bin records per
 *      row) as wedge_sample_close.
 *      h_info         nullable host uint64[4]: m (edges counted), edges
 *                     skipped for an id >= n, gather rounds, edge ends
 *                     gathered.
 * Workspace: wedge_sample_stream_workspace(n, m_in, max_bins, h_k, k_global,
 *            gather_cap, chunk_edges) bytes (256-byte aligned).
 * Unlike the other calls this one synchronises `stream` (it sizes later
 * passes from earlier results).
 * Errors: EINVAL, ERANGE (n == 0, tau == 0, omega < 2, max_bins outside
 *         [1, 4096], gather_cap outside [1, 2^40), a k above 2^40),
 *         EWORKSPACE (workspace, or a drawn centre's degree above
 *         gather_cap), EGRAPH (repeated edges found in a drawn centre's
 *         row; the results are then not those of the simple graph), EHIP.
 * ---------------------------------------------------------------------- */
size_t wedge_sample_stream_workspace(uint32_t n, uint64_t m_in, uint32_t max_bins,
                                     const uint64_t* h_k, uint64_t k_global,
                                     uint64_t gather_cap, uint64_t chunk_edges);
int wedge_sample_stream(const uint32_t* h_src, const uint32_t* h_dst, uint64_t m_in, uint32_t n,
                        uint32_t tau, uint64_t omega, uint32_t max_bins, const uint64_t* h_k,
                        uint64_t k_global, uint64_t seed, uint64_t gather_cap,
                        uint64_t chunk_edges, uint64_t* d_n_b, uint64_t* d_p_b, uint64_t* d_q,
                        wedge_sample_rec* d_dump, uint64_t dump_per_bin, uint64_t* h_info,
                        void* d_workspace, size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Triangle sample and degree assortativity (Sec. 3 theorem on sampled
 * triangles; Sec. 5 triangle statistics).  A closed wedge of a uniform wedge
 * sample is a uniform sample (with replacement) of the graph's triangles,
 * since every triangle owns exactly three wedges.  The global stream (row
 * max_bins) draws wedges uniformly from the whole graph, so its closed
 * records are uniform triangles; the paper obtains the same with one bin
 * (tau = 1, omega = 10^7).
 *
 * In:  d_rec[k]  feature records of one row (wedge_sample_features with
 *                closure = 1; WEDGE_DOMAIN_SAMPLE reproduces the samples of
 *                wedge_sample_close), k < 2^32.
 * Out: d_tri     nullable wedge_triangle[k]: the closed records' degree
 *                triples in record order (compacted: triangle j is the j-th
 *                closed record); entries past the count are untouched.
 *      d_count   device uint64[1]: number of closed records.
 *      d_hist    device uint64[max_bins * max_bins], overwritten:
 *                d_hist[BinId(d_min) * max_bins + BinId(d_max)] counts the
 *                triangles, BinId with (tau, omega) (the paper groups with
 *                tau = omega = 2); a triangle whose BinId(d_max) >= max_bins
 *                is counted in d_count only.
 * Workspace: wedge_triangle_stats_workspace(k) bytes.
 * Errors: EINVAL, ERANGE (k >= 2^32, max_bins == 0 or > 64, tau == 0,
 *         omega < 2), EWORKSPACE, EHIP.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint32_t d_min, d_mid, d_max; /* degrees of the triangle's vertices, sorted */
  uint32_t sample;              /* index of its record in d_rec */
} wedge_triangle;

size_t wedge_triangle_stats_workspace(uint64_t k);
int wedge_triangle_stats(const wedge_feature_rec* d_rec, uint64_t k, uint32_t tau,
                         uint64_t omega, uint32_t max_bins, wedge_triangle* d_tri,
                         uint64_t* d_count, uint64_t* d_hist, void* d_workspace,
                         size_t workspace_bytes, void* stream);

/* Box-plot statistics of the max-degree bin of the triangles in each
 * min-degree bin, from a host copy of d_hist (host only).  Percentiles are
 * nearest-rank: the p-quantile of N values is the smallest bin b with at
 * least ceil(p N) of them <= b; whiskers are the most extreme bins within
 * 1.5 IQR of the quartiles (Tukey), outliers the triangles beyond them.
 * h_out[max_bins]: row b describes the triangles whose BinId(d_min) = b
 * (count 0: none). */
typedef struct {
  uint64_t count;
  uint64_t outliers;
  uint32_t q1, median, q3;
  uint32_t whisker_lo, whisker_hi;
  uint32_t pad;
} wedge_triangle_box_row;

int wedge_triangle_box(const uint64_t* h_hist, uint32_t max_bins, wedge_triangle_box_row* h_out);

/* ------------------------------------------------------------------------
 * Control-variate estimator (host-only arithmetic; the estimand is c_b of
 * Thm. cd-est).  Inputs are the integer moments of wedge_cv_moments,
 * m = [count, sum X, 2^32 sum g, 2^32 sum g^2, 2^32 sum X g].  With
 * n = m[0], mx = m[1]/n, mg = m[2]/2^32/n and (n - 1)-denominator
 *   var_x = (m[1] - n mx^2)/(n-1),  var_g = (m[3]/2^32 - n mg^2)/(n-1),
 *   cov   = (m[4]/2^32 - n mx mg)/(n-1),  var_z = var_x - 2 beta cov + beta^2 var_g,
 * the estimate of a row is mean(X - beta g) + beta mu = mx - beta mg + beta mu.
 * ---------------------------------------------------------------------- */

/* Empirical-Bernstein half-width (Maurer & Pontil 2009, Thm. 4, two-sided,
 * each side at delta/2) of the mean of n i.i.d. values in an interval of
 * length R with sample variance var (negative var taken as 0):
 *   sqrt(2 var ln(4/delta) / n) + 7 R ln(4/delta) / (3 (n - 1)).
 * Host-only; returns +inf for n < 2. */
double wedge_eb_halfwidth(uint64_t n, double var, double R, double delta);

/* Planning size for that bound to reach eps: with n - 1 taken as n, the
 * positive root x = 1/sqrt(n) of a x + b x^2 = eps, a = sqrt(2 var ln(4/delta)),
 * b = 7 R ln(4/delta) / 3; returns ceil(1/x^2) + 1 (0 for eps <= 0, R <= 0
 * or delta outside (0, 1)).  A plan only: stopping uses the exact bound. */
uint64_t wedge_eb_samples(double var, double R, double delta, double eps);

/* Running total of a row's draws after round `round` >= 1 of a plan that
 * starts at `first` and grows by `growth` per round:
 * min(ceil(first growth^(round-1)), max_per_row); 0 for round 0. */
uint64_t wedge_cv_round_size(uint64_t first, double growth, uint32_t round,
                             uint64_t max_per_row);

/* Fit of the control variate per row from held-out TRAIN moments (h_mom
 * [rows][5]): beta = Cov(X, g) / Var(g) and rho^2 = Cov^2 / (Var X Var g) from
 * n-denominator moments (0 when Var g <= 1e-14 or n < 2), var_x and var_z
 * ((n - 1) denominators; 0.25 each when n < 2), and the first-round sizes
 * wedge_eb_samples at delta / 2 for plain sampling (var_x, range 1) and for
 * the control variate (var_z, range 1 + |beta|).  The fit uses no EVAL draw,
 * so the estimate stays unbiased.  Errors: EINVAL. */
typedef struct {
  double beta, rho2, var_x, var_z;
  uint64_t plan_plain, plan_cv;
} wedge_cv_fit_row;
int wedge_cv_fit(const int64_t* h_mom, uint32_t rows, double eps, double delta,
                 wedge_cv_fit_row* h_out);

/* Where the mean mu of g comes from. */
enum { WEDGE_CV_PLAIN = 0,   /* beta ignored: the plain mean of X, range 1 */
       WEDGE_CV_EXACT = 1,   /* mu = exact_mean (census): whole delta_i on the EVAL draws */
       WEDGE_CV_AUX = 2,     /* mu = mean of g over AUX draws (an, ag, ag2) */
       WEDGE_CV_CENTRE = 3   /* mu = mean of gbar over centre draws (an, ag, ag2);
                                beta = 0 is the plain form */ };

typedef struct {
  int64_t n, sx, sg, sg2, sxg;   /* EVAL moments accumulated so far */
  int64_t an, ag, ag2;           /* second sample: count, 2^32 sum, 2^32 sum of squares */
  double beta;                   /* fixed before any EVAL draw */
  double exact_mean;             /* WEDGE_CV_EXACT only */
  uint32_t mode;                 /* WEDGE_CV_* */
  uint32_t pad;
  uint64_t done;                 /* EVAL draws taken so far (checked against the cap) */
} wedge_cv_row;

typedef struct {
  double estimate;   /* NaN when a sample has fewer than 2 draws */
  double halfwidth;  /* +inf then */
  int32_t more;      /* 1: halfwidth > eps and done < max_per_row */
  int32_t pad;
} wedge_cv_result;

/* Estimate, half-width and stop decision of every row after round `round`
 * (>= 1) of the sequential rule: delta_i = delta / (round (round + 1)) (a
 * union bound over rounds).  PLAIN: mx, EB(n, var_x, 1, delta_i).  EXACT:
 * mx - beta mg + beta exact_mean, EB(n, var_z, 1 + |beta|, delta_i).  AUX and
 * CENTRE (beta != 0): mx - beta mg + beta am with am, av the mean and
 * (an - 1)-denominator variance of the second sample,
 * EB(n, var_z, 1 + |beta|, delta_i/2) + |beta| EB(an, av, 1, delta_i/2).
 * Errors: EINVAL (null pointer, round 0, eps <= 0, delta outside (0,1),
 * unknown mode). */
int wedge_cv_estimate(const wedge_cv_row* h_rows, uint32_t nrows, uint32_t round, double delta,
                      double eps, uint64_t max_per_row, wedge_cv_result* h_out);

/* Exact mean of g per bin from the per-key sums of wedge_cv_exact_mean:
 * h_mean[b] = (sum of h_key_sum over keys of bin b) / (their wedge counts),
 * summed in key order; h_mean[max_bins] = the same over every key (the
 * global stream's mean); h_count[b] = wedges of the bin (p_b), and
 * h_count[max_bins] = p.  Bins without keys get mean 0 and count 0.
 * Errors: EINVAL (null pointer, a key's bin >= max_bins). */
int wedge_cv_bin_means(const double* h_key_sum, const uint64_t* h_key_count,
                       const uint32_t* h_key_bin, uint32_t nkeys, uint32_t max_bins,
                       double* h_mean, uint64_t* h_count);

/* Mean (2^32 sum / count; NaN for count 0) and (n - 1)-denominator variance
 * (0 for count < 2, negative taken as 0) of the values whose moments are
 * h_mom[rows][5] (entries 0, 2, 3 used). */
int wedge_cv_mean_var(const int64_t* h_mom, uint32_t rows, double* h_mean, double* h_var);

/* Modelled cost of one centre draw of row `row` (a bin < max_bins, or the
 * global stream = max_bins) in EVAL draws: 1 + a d^b with d the degree whose
 * C(d, 2) is the row's mean wedges per vertex (0.5 + sqrt(0.25 + 2 p_b / n_b));
 * the global row averages the bins' d weighted by p_b. */
double wedge_cv_centre_cost(const uint64_t* h_n_b, const uint64_t* h_p_b, uint32_t max_bins,
                            uint32_t row, double a, double b);

/* First-round plan of the centre form per row: with the fit, the variance
 * of gbar from a pilot (h_centre_var) and the cost per centre draw (h_cost),
 * the share t in {0.01, ..., 0.99} of eps given to the centre term that
 * minimises wedge_eb_samples(var_z, 1+|beta|, delta/4, eps (1-t)) + cost
 * wedge_eb_samples(var, 1, delta/4, eps t/|beta|); if that is not below the
 * plain plan wedge_eb_samples(var_x, 1, delta/2, eps), or beta = 0, the row
 * stays plain (h_centre = 0, h_beta = 0).  Outputs per row: EVAL draws,
 * centre draws, beta used. */
int wedge_cv_plan_centre(const wedge_cv_fit_row* h_fit, const double* h_centre_var,
                         const double* h_cost, uint32_t rows, double eps, double delta,
                         uint64_t* h_eval, uint64_t* h_centre, double* h_beta);

/* Training of the control variate on TRAIN draws (key domain 2) of the rows
 * h_rows[nrows] (increasing, bins < max_bins and/or the global stream
 * max_bins): draws 0 .. n_fit - 1 of every row fit the network (fan-in
 * initialisation from init_seed, then `epochs` passes of Adam on minibatches
 * of per_row_batch draws of every row, lr, beta1 0.9, beta2 0.999, eps 1e-8),
 * draws n_fit .. n_fit + n_hold - 1 are held out: their moments (h_mom
 * [nrows][5], nullable) give h_fit[nrows] as wedge_cv_fit does.  h_loss
 * (nullable): the last minibatch's mean loss.  d_state: the network state,
 * trained in place.  Synchronises the stream (it reads the moments back).
 * Workspace: wedge_cv_train_workspace(nrows, n_fit, n_hold, per_row_batch).
 * Errors: EINVAL, ERANGE (max_bins > 4096), EWORKSPACE, and those of the
 * calls it makes. */
size_t wedge_cv_train_workspace(uint32_t rows, uint64_t n_fit, uint64_t n_hold,
                                uint64_t per_row_batch);
int wedge_cv_train(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n, uint64_t m,
                   const void* d_index, uint32_t max_bins, uint32_t tau, uint64_t omega,
                   const uint32_t* h_rows, uint32_t nrows, uint64_t n_fit, uint64_t n_hold,
                   uint64_t per_row_batch, uint32_t epochs, float lr, uint64_t seed,
                   uint64_t init_seed, void* d_state, double eps, double delta,
                   wedge_cv_fit_row* h_fit, int64_t* h_mom, float* h_loss, void* d_workspace,
                   size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* WEDGE_H */
