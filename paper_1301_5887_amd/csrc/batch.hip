// Batched form: many graphs of uneven size and all their degree bins in one
// pass of each kernel, with no host round trip, so the whole pipeline can be
// captured once into a HIP graph and replayed.
//
// The graphs of a batch become one block-diagonal CSR (vertex ids shifted by
// each graph's vertex offset), so a single sort builds every adjacency; the
// sampling index carries a graph dimension (rows g * (max_bins + 1) + bin);
// a planning scan turns the per-row wedge counts into a device task table of
// (row, samples, first tile), and one persistent sampler grid drains the
// tiles of every row of every graph from a ticket counter.  Per-graph
// estimates (Alg. phase4c, Eq. global_est) are computed on the device in
// FP64 in the same operation order as the host summary.
#include <math.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "rng.hpp"
#include "sample.hpp"
#include "scan.hpp"

namespace wedge {

struct BatchLayout {
  uint64_t* rowptr;
  uint32_t* col;
  uint64_t* info;
  void* index;
  uint64_t* task_k;
  uint64_t* tile_begin;
  unsigned long long* ticket;
  unsigned int* flag;
  void* scratch;
};

static uint64_t batch_rows(const wedge_batch_desc* d) {
  return (uint64_t)d->num_graphs * ((uint64_t)d->max_bins + 1);
}

static size_t batch_layout(const wedge_batch_desc* d, BatchLayout* L, void* base) {
  const uint64_t n = d->total_vertices, m_in = d->total_edges;
  const uint32_t G = d->num_graphs, B = d->max_bins;
  const uint64_t rows = batch_rows(d);
  char* c = (char*)base;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = c ? c + off : nullptr;  // sizing calls pass no base
    off += round_up(bytes ? bytes : 1, 256);
    return (void*)p;
  };
  void* rp = take((n + 1) * 8);
  void* cl = take((m_in ? 2 * m_in : 1) * 4);
  void* inf = take(16);
  void* ix = take(index_bytes(n, m_in, G, B));
  void* tk = take(rows * 8);
  void* tb = take((rows + 1) * 8);
  void* tkt = take(8);
  void* flg = take(8);
  size_t scratch = csr_workspace_bytes(m_in);
  const size_t bw = bins_workspace_bytes(n, G, B);
  if (bw > scratch) scratch = bw;
  const size_t sw = scan_ws_elems(rows) * 8;
  if (sw > scratch) scratch = sw;
  void* scr = take(scratch);
  if (L) {
    L->rowptr = (uint64_t*)rp;
    L->col = (uint32_t*)cl;
    L->info = (uint64_t*)inf;
    L->index = ix;
    L->task_k = (uint64_t*)tk;
    L->tile_begin = (uint64_t*)tb;
    L->ticket = (unsigned long long*)tkt;
    L->flag = (unsigned int*)flg;
    L->scratch = scr;
  }
  return off;
}

static int check_desc(const wedge_batch_desc* d) {
  if (!d) return set_error(WEDGE_EINVAL, "batch: null descriptor");
  if (d->num_graphs == 0) return set_error(WEDGE_ERANGE, "batch: num_graphs must be >= 1");
  if (d->max_bins == 0 || d->max_bins > 4096)
    return set_error(WEDGE_ERANGE, "batch: max_bins must be in [1, 4096]");
  if (d->tau == 0 || d->omega < 2)
    return set_error(WEDGE_ERANGE, "batch: need tau >= 1 and integer omega >= 2");
  if (d->total_vertices == 0 || d->max_n == 0 || d->max_n > d->total_vertices)
    return set_error(WEDGE_ERANGE, "batch: inconsistent vertex counts");
  if (d->total_vertices >= (1ULL << 32))
    return set_error(WEDGE_ERANGE, "batch: total_vertices must be < 2^32");
  if (d->total_edges >= (1ULL << 40)) return set_error(WEDGE_ERANGE, "batch: total_edges >= 2^40");
  const int gbits = d->num_graphs > 1 ? bit_width((uint64_t)d->num_graphs - 1) : 0;
  if (gbits > 0 && (uint64_t)d->max_n > (1ULL << (32 - gbits)))
    return set_error(WEDGE_ERANGE, "batch: max_n above 2^%d for %u graphs", 32 - gbits,
                     d->num_graphs);
  if (d->k_per_bin > (1ULL << 48) || d->k_global > (1ULL << 48))
    return set_error(WEDGE_ERANGE, "batch: k above 2^48");
  return WEDGE_OK;
}

struct PlanK {
  const BinMeta* bins;
  uint32_t B;
  uint64_t k_bin, k_glob;
  __device__ uint64_t k(uint64_t f) const {
    const uint32_t row = (uint32_t)(f % (B + 1));
    return bins[f].p_b > 0 ? (row == B ? k_glob : k_bin) : 0;
  }
};

struct PlanLoad {
  PlanK pk;
  uint64_t spt;
  __device__ uint64_t operator()(uint64_t f) const { return (pk.k(f) + spt - 1) / spt; }
};

struct PlanApply {
  PlanK pk;
  uint64_t rows;
  uint64_t* task_k;
  uint64_t* tile_begin;
  __device__ void operator()(uint64_t f, uint64_t prefix, uint64_t tiles) const {
    task_k[f] = pk.k(f);
    tile_begin[f] = prefix;
    if (f == rows - 1) tile_begin[rows] = prefix + tiles;
  }
};

// Per graph, in the order of the host summary: bins ascending, then the
// weighted global estimate and the global stream.  lg = ln(2/delta) is
// computed once on the host so both sides use the same value.
__global__ void k_batch_estimate(const BinMeta* __restrict__ bins, const uint64_t* __restrict__ q,
                                 const uint64_t* __restrict__ task_k, uint32_t G, uint32_t B,
                                 double lg, double* __restrict__ est_glob,
                                 double* __restrict__ est_bins) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const uint64_t r0 = (uint64_t)g * (B + 1);
  uint64_t p = 0;
  for (uint32_t b = 0; b < B; ++b) p += bins[r0 + b].p_b;
  double num = 0.0, tsum = 0.0;
  for (uint32_t b = 0; b < B; ++b) {
    const uint64_t f = r0 + b;
    const uint64_t k = task_k[f];
    const uint64_t* qb = q + f * 4;
    const uint64_t pb = bins[f].p_b;
    double c = 0.0, t = 0.0, e = 0.0;
    if (k > 0) {
      c = (double)(qb[1] + qb[2] + qb[3]) / (double)k;
      const uint64_t t6 = 6 * qb[1] + 3 * qb[2] + 2 * qb[3];
      t = ((double)pb * (double)t6) / (6.0 * (double)k);
      e = sqrt(lg / (2.0 * (double)k));
    }
    if (est_bins) {
      est_bins[((uint64_t)g * B + b) * 3 + 0] = c;
      est_bins[((uint64_t)g * B + b) * 3 + 1] = t;
      est_bins[((uint64_t)g * B + b) * 3 + 2] = e;
    }
    num += (double)pb * c;
    tsum += t;
  }
  const double cw = p > 0 ? num / (double)p : 0.0;
  const uint64_t fg = r0 + B;
  const uint64_t kg = task_k[fg];
  const double cg = kg > 0 ? (double)q[fg * 4 + 3] / (double)kg : 0.0;
  if (est_glob) {
    est_glob[(uint64_t)g * 6 + 0] = cw;
    est_glob[(uint64_t)g * 6 + 1] = cw * (double)p / 3.0;
    est_glob[(uint64_t)g * 6 + 2] = cg;
    est_glob[(uint64_t)g * 6 + 3] = cg * (double)p / 3.0;
    est_glob[(uint64_t)g * 6 + 4] = kg > 0 ? sqrt(lg / (2.0 * (double)kg)) : 0.0;
    est_glob[(uint64_t)g * 6 + 5] = tsum;
  }
}

static int batch_prepare_impl(const wedge_batch_desc* d, const uint32_t* d_src,
                              const uint32_t* d_dst, const uint64_t* d_eoff,
                              const uint32_t* d_voff, uint64_t* d_n_b, uint64_t* d_p_b,
                              void* d_ws, hipStream_t st) {
  BatchLayout L;
  batch_layout(d, &L, d_ws);
  int rc = csr_build(d_src, d_dst, d->total_edges, d->total_vertices, d_eoff, d_voff,
                     d->num_graphs, L.rowptr, L.col, L.info, L.scratch, st);
  if (rc) return rc;
  return bins_build(L.rowptr, d->total_vertices, d->total_edges, d_voff, d->num_graphs,
                    d->max_n, d->tau, d->omega, d->max_bins, d_n_b, d_p_b, L.index, L.scratch,
                    st);
}

static int batch_sample_impl(const wedge_batch_desc* d, const SampleTuning* shape, double delta,
                             uint64_t* d_q, uint64_t* d_probe_loads, double* d_est_glob,
                             double* d_est_bins, void* d_ws, hipStream_t st) {
  BatchLayout L;
  batch_layout(d, &L, d_ws);
  const uint64_t rows = batch_rows(d);
  // typical sample count: every graph samples about bits(max_n) + 2 bins
  const uint64_t approx = (uint64_t)d->num_graphs *
                          ((uint64_t)(bit_width(d->max_n) + 2) * d->k_per_bin + d->k_global);
  SampleTuning t = shape ? *shape : default_tuning(approx);
  normalise(t);
  SamplerCtx A;
  A.rowptr = L.rowptr;
  A.col = L.col;
  A.ix = index_view(L.index, d->total_vertices, d->total_edges, d->num_graphs, d->max_bins);
  A.seed = d->seed;
  A.spt = t.spt;
  A.dump_per_bin = 0;
  A.q = d_q;
  A.probe_loads = d_probe_loads;
  A.dump = nullptr;
  A.class_cap = class_capacity(d->total_vertices, d->total_edges, d->num_graphs);
  A.n = d->total_vertices;
  A.max_bins = d->max_bins;
  A.num_graphs = d->num_graphs;
  A.domain = kDomainSample;
  A.s_begin = 0;
  A.feat = nullptr;
  A.feat_stride = 0;
  A.omega = d->omega;
  A.tau = d->tau;
  A.closure = 1;
  int rc;
  if ((rc = fill<uint64_t>(d_q, rows * 4, 0, st))) return rc;
  if (d_probe_loads && (rc = fill<uint64_t>(d_probe_loads, 1, 0, st))) return rc;
  PlanK pk{A.ix.bins, d->max_bins, d->k_per_bin, d->k_global};
  rc = scan_apply<uint64_t>(PlanLoad{pk, t.spt}, PlanApply{pk, rows, L.task_k, L.tile_begin}, rows,
                            (uint64_t*)L.scratch, st);
  if (rc) return rc;
  rc = launch_persistent(A, L.task_k, L.tile_begin, rows, L.ticket, t, st);
  if (rc) return rc;
  if (d_est_glob || d_est_bins) {
    k_batch_estimate<<<(unsigned)ceil_div(d->num_graphs, 64), 64, 0, st>>>(
        A.ix.bins, d_q, L.task_k, d->num_graphs, d->max_bins, log(2.0 / delta), d_est_glob,
        d_est_bins);
    WEDGE_LAUNCH_CHECK("k_batch_estimate");
  }
  return WEDGE_OK;
}

static SampleTuning from_shape(const wedge_launch_shape* s) {
  SampleTuning t{4, 4096, 0};
  if (s) {
    t.U = s->lanes_in_flight;
    t.spt = s->samples_per_tile;
    t.workgroups = s->workgroups;
  }
  return t;
}

struct BatchGraph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

__global__ void k_compare_u64(const uint64_t* a, const uint64_t* b, uint64_t n,
                              unsigned int* differ) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride)
    if (a[i] != b[i]) atomicOr(differ, 1u);
}

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_batch_workspace_bytes(const wedge_batch_desc* d) {
  if (!d || check_desc(d) != WEDGE_OK) return 0;
  return batch_layout(d, nullptr, nullptr);
}

extern "C" int wedge_batch_prepare(const wedge_batch_desc* d, const uint32_t* d_src,
                                   const uint32_t* d_dst, const uint64_t* d_edge_off,
                                   const uint32_t* d_vert_off, uint64_t* d_n_b, uint64_t* d_p_b,
                                   void* d_workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!d_edge_off || !d_vert_off || !d_n_b || !d_p_b || !d_workspace ||
      (d->total_edges > 0 && (!d_src || !d_dst)))
    return set_error(WEDGE_EINVAL, "wedge_batch_prepare: null pointer");
  if (!aligned(d_workspace, 256) || !aligned(d_edge_off, 8) || !aligned(d_vert_off, 4) ||
      !aligned(d_n_b, 8) || !aligned(d_p_b, 8))
    return set_error(WEDGE_EINVAL, "wedge_batch_prepare: misaligned pointer");
  if (workspace_bytes < batch_layout(d, nullptr, nullptr))
    return set_error(WEDGE_EWORKSPACE, "wedge_batch_prepare: workspace too small");
  return batch_prepare_impl(d, d_src, d_dst, d_edge_off, d_vert_off, d_n_b, d_p_b, d_workspace,
                            (hipStream_t)stream);
}

extern "C" int wedge_batch_sample(const wedge_batch_desc* d, const wedge_launch_shape* shape,
                                  double delta, uint64_t* d_q, uint64_t* d_probe_loads,
                                  double* d_est_glob, double* d_est_bins, void* d_workspace,
                                  size_t workspace_bytes, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!d_q || !d_workspace) return set_error(WEDGE_EINVAL, "wedge_batch_sample: null pointer");
  if (!(delta > 0.0) || !(delta < 1.0))
    return set_error(WEDGE_EINVAL, "wedge_batch_sample: delta must be in (0, 1)");
  if (!aligned(d_workspace, 256) || !aligned(d_q, 8) || !aligned(d_probe_loads, 8) ||
      !aligned(d_est_glob, 8) || !aligned(d_est_bins, 8))
    return set_error(WEDGE_EINVAL, "wedge_batch_sample: misaligned pointer");
  if (workspace_bytes < batch_layout(d, nullptr, nullptr))
    return set_error(WEDGE_EWORKSPACE, "wedge_batch_sample: workspace too small");
  SampleTuning t = from_shape(shape);
  return batch_sample_impl(d, shape ? &t : nullptr, delta, d_q, d_probe_loads, d_est_glob,
                           d_est_bins, d_workspace, (hipStream_t)stream);
}

extern "C" int wedge_batch_run(const wedge_batch_desc* d, const uint32_t* d_src,
                               const uint32_t* d_dst, const uint64_t* d_edge_off,
                               const uint32_t* d_vert_off, const wedge_launch_shape* shape,
                               double delta, uint64_t* d_n_b, uint64_t* d_p_b, uint64_t* d_q,
                               double* d_est_glob, double* d_est_bins, void* d_workspace,
                               size_t workspace_bytes, void* stream) {
  int rc = wedge_batch_prepare(d, d_src, d_dst, d_edge_off, d_vert_off, d_n_b, d_p_b, d_workspace,
                               workspace_bytes, stream);
  if (rc) return rc;
  return wedge_batch_sample(d, shape, delta, d_q, nullptr, d_est_glob, d_est_bins, d_workspace,
                            workspace_bytes, stream);
}

extern "C" int wedge_batch_graph_create(const wedge_batch_desc* d, const uint32_t* d_src,
                                        const uint32_t* d_dst, const uint64_t* d_edge_off,
                                        const uint32_t* d_vert_off,
                                        const wedge_launch_shape* shape, double delta,
                                        uint64_t* d_n_b, uint64_t* d_p_b, uint64_t* d_q,
                                        double* d_est_glob, double* d_est_bins,
                                        void* d_workspace, size_t workspace_bytes,
                                        void** h_graph) {
  clear_error();
  if (!h_graph) return set_error(WEDGE_EINVAL, "wedge_batch_graph_create: null out-pointer");
  *h_graph = nullptr;
  hipStream_t cs;
  WEDGE_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    hipStreamDestroy(cs);
    return set_error(WEDGE_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  int rc = wedge_batch_run(d, d_src, d_dst, d_edge_off, d_vert_off, shape, delta, d_n_b, d_p_b,
                           d_q, d_est_glob, d_est_bins, d_workspace, workspace_bytes, cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  hipStreamDestroy(cs);
  if (rc) {
    if (graph) hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return set_error(WEDGE_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(graph);
    return set_error(WEDGE_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *h_graph = new BatchGraph{graph, exec};
  return WEDGE_OK;
}

extern "C" int wedge_batch_graph_launch(void* h_graph, void* stream) {
  clear_error();
  if (!h_graph) return set_error(WEDGE_EINVAL, "wedge_batch_graph_launch: null graph");
  WEDGE_HIP_TRY(hipGraphLaunch(((BatchGraph*)h_graph)->exec, (hipStream_t)stream));
  return WEDGE_OK;
}

extern "C" int wedge_batch_graph_destroy(void* h_graph) {
  clear_error();
  if (!h_graph) return WEDGE_OK;
  BatchGraph* g = (BatchGraph*)h_graph;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
  return WEDGE_OK;
}

// Autotuner: times every candidate launch shape of the batch sampler on the
// prepared batch (median of `reps` runs, HIP events on `stream`), checks that
// each candidate's class counts equal the first candidate's bit for bit, and
// reports the fastest.
extern "C" int wedge_batch_autotune(const wedge_batch_desc* d, const wedge_launch_shape* cands,
                                    int ncand, int reps, uint64_t* d_q_ref, uint64_t* d_q_try,
                                    void* d_workspace, size_t workspace_bytes, float* h_ms,
                                    int* h_best, void* stream) {
  clear_error();
  int rc = check_desc(d);
  if (rc) return rc;
  if (!cands || ncand <= 0 || reps <= 0 || !d_q_ref || !d_q_try || !h_ms || !h_best)
    return set_error(WEDGE_EINVAL, "wedge_batch_autotune: bad arguments");
  if (workspace_bytes < batch_layout(d, nullptr, nullptr))
    return set_error(WEDGE_EWORKSPACE, "wedge_batch_autotune: workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const uint64_t nq = batch_rows(d) * 4;
  BatchLayout L;
  batch_layout(d, &L, d_workspace);
  unsigned int* d_diff = L.flag;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  int best = -1;
  for (int c = 0; c < ncand && rc == WEDGE_OK; ++c) {
    std::vector<float> t(reps);
    uint64_t* q = c == 0 ? d_q_ref : d_q_try;
    for (int r = 0; r < reps && rc == WEDGE_OK; ++r) {
      hipEventRecord(e0, st);
      rc = wedge_batch_sample(d, &cands[c], 0.5, q, nullptr, nullptr, nullptr, d_workspace,
                              workspace_bytes, st);
      hipEventRecord(e1, st);
      hipEventSynchronize(e1);
      hipEventElapsedTime(&t[r], e0, e1);
    }
    if (rc) break;
    std::sort(t.begin(), t.end());
    h_ms[c] = t[reps / 2];
    if (c > 0) {
      unsigned int diff = 0;
      if ((rc = fill<unsigned int>(d_diff, 1, 0u, st))) break;
      k_compare_u64<<<256, 256, 0, st>>>(d_q_ref, d_q_try, nq, d_diff);
      const hipError_t e1 = hipMemcpyAsync(&diff, d_diff, sizeof(diff), hipMemcpyDeviceToHost, st);
      const hipError_t e2 = hipStreamSynchronize(st);  // also when the copy was refused
      if (e1 != hipSuccess || e2 != hipSuccess) {
        rc = set_error(WEDGE_EHIP, "wedge_batch_autotune: reading the comparison failed: %s",
                       hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        break;
      }
      if (diff) {
        rc = set_error(WEDGE_EINVAL, "wedge_batch_autotune: counts of candidate %d differ", c);
        break;
      }
    }
    if (best < 0 || h_ms[c] < h_ms[best]) best = c;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  *h_best = best;
  return WEDGE_OK;
}
