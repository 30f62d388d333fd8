// Sampler launch interface shared by the single-graph and batched paths.
#pragma once

#include "common.hpp"

namespace wedge {

constexpr int kSampWG = 256;
constexpr int kMaxTasks = 64;

// Allocation form (Alg. phase2a): row f's vertices are vlist positions
// [pos_lo, pos_lo + count); their sample counts sit at [off, off + count) of
// a concatenated array whose exclusive prefix (alloc_pre) numbers the row's
// samples, so sample s of the row is centred at the vertex whose prefix
// range holds alloc_pre[off] + s.
struct AllocRow {
  uint64_t off;
  uint64_t count;
  uint64_t pos_lo;
  uint64_t k;
};

// Everything a tile needs, passed by value to the kernels.
struct SamplerCtx {
  const uint64_t* rowptr;
  const uint32_t* col;
  IndexView ix;
  uint64_t seed;
  uint64_t spt;  // samples per tile
  uint64_t dump_per_bin;
  uint64_t* q;   // [rows * 4], row f = g * (max_bins + 1) + bin
  uint64_t* probe_loads;
  wedge_sample_rec* dump;
  uint64_t class_cap;
  uint32_t n;
  uint32_t max_bins;
  uint32_t num_graphs;
  // stream selection and the feature output of the control variate
  uint64_t domain;        // Philox key word 1 (1 = plain sampling)
  uint64_t s_begin;       // first sample index of every row (persistent form)
  wedge_feature_rec* feat;  // nullable: record of sample s of a task at
  uint64_t feat_stride;     //   slot * feat_stride + (s - the task's s_begin)
  uint64_t omega;           // binning, for the centre's bin in a record
  uint32_t tau;
  int closure;              // 0: skip the closure search (feature-only draws)
  // allocation form: centres from per-vertex counts instead of word 0
  const AllocRow* alloc = nullptr;     // [rows], nullable
  const uint64_t* alloc_pre = nullptr; // exclusive prefix of the counts
  // closure by lookup in the edge table of hash.hpp instead of the search
  const uint64_t* hash = nullptr;      // nullable
  int hash_bits = 0;
  // draws only: the dump receives (centre, i, j, 0) of every sample and no
  // adjacency is read (the streamed path resolves i, j later)
  int draw_only = 0;
};

struct Task {
  uint32_t row;    // index row (bin id, or max_bins for the global stream)
  uint32_t bword;  // Philox counter word 1: bin id, or 0xFFFFFFFF
  uint64_t k;      // samples s_begin .. s_begin + k - 1
  uint64_t s_begin;
  uint64_t tile_begin;
  uint64_t slot;   // feature-record row of this task
};

struct TaskTable {
  uint64_t graph_word;  // Philox counter word 2
  uint32_t ntask;
  Task task[kMaxTasks];
};

// Launch shape: samples carried per lane (1, 2, 4, 8), samples per tile, and
// workgroups of the persistent grid.
struct SampleTuning {
  int U;
  uint64_t spt;
  uint32_t workgroups;
};

SampleTuning default_tuning(uint64_t total_samples);
void normalise(SampleTuning& t);

// Draws only (see SamplerCtx::draw_only) of wedge_sample_close's samples:
// record s of row r (bin r, or max_bins for the global stream) goes to
// d_rec[r * stride + s] for every s < h_k[r] (k_global for the global row);
// stride must be >= every row's k.  Only rowptr (degrees) and the index are
// read; d_q ((max_bins + 1) * 4 uint64) is cleared and left at zero.
int sample_draws(const uint64_t* d_rowptr, uint32_t n, uint64_t m, const void* d_index,
                 uint32_t max_bins, const uint64_t* h_k, uint64_t k_global, uint64_t seed,
                 wedge_sample_rec* d_rec, uint64_t stride, uint64_t* d_q, hipStream_t st);

int launch_persistent(const SamplerCtx& A, const uint64_t* task_k, const uint64_t* tile_begin,
                      uint64_t nrows, unsigned long long* ticket, const SampleTuning& t,
                      hipStream_t st);

}  // namespace wedge
