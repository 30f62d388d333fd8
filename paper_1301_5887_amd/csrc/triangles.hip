// Triangle sample and degree assortativity: the closed records among
// uniform wedge samples are uniform triangles (every triangle owns three
// wedges, Sec. 3); each is reduced to its sorted vertex degrees and counted
// by (BinId(d_min), BinId(d_max)) for the assortativity statistics of Sec. 5.
//
// One exclusive scan over the closed flags numbers the triangles in record
// order; its consumer writes triangle j at its position and adds it to the
// histogram, so the compaction costs one read of the records.
#include "common.hpp"
#include "scan.hpp"

namespace wedge {

struct TriLoad {
  const wedge_feature_rec* rec;
  __device__ uint64_t operator()(uint64_t i) const { return rec[i].closed ? 1 : 0; }
};

struct TriApply {
  const wedge_feature_rec* rec;
  wedge_triangle* tri;
  uint64_t* hist;
  uint64_t* count;
  uint64_t k;
  uint64_t omega;
  uint32_t tau;
  uint32_t max_bins;
  __device__ void operator()(uint64_t i, uint64_t prefix, uint64_t x) const {
    if (x) {
      const wedge_feature_rec r = rec[i];
      // dlo <= dhi already; place the centre's degree among them
      const uint32_t lo = r.dv < r.dlo ? r.dv : r.dlo;
      const uint32_t hi = r.dv > r.dhi ? r.dv : r.dhi;
      const uint32_t mid = r.dv < r.dlo ? r.dlo : (r.dv > r.dhi ? r.dhi : r.dv);
      if (tri) tri[prefix] = wedge_triangle{lo, mid, hi, (uint32_t)i};
      const uint32_t b0 = bin_id_capped(lo, tau, omega, max_bins);
      const uint32_t b1 = bin_id_capped(hi, tau, omega, max_bins);
      if (b1 < max_bins)
        atomicAdd((unsigned long long*)&hist[(uint64_t)b0 * max_bins + b1], 1ULL);
    }
    if (i == k - 1) *count = prefix + x;
  }
};

}  // namespace wedge

using namespace wedge;

extern "C" size_t wedge_triangle_stats_workspace(uint64_t k) {
  return round_up(scan_ws_elems(k) * 8, 256);
}

extern "C" int wedge_triangle_stats(const wedge_feature_rec* d_rec, uint64_t k, uint32_t tau,
                                    uint64_t omega, uint32_t max_bins, wedge_triangle* d_tri,
                                    uint64_t* d_count, uint64_t* d_hist, void* d_workspace,
                                    size_t workspace_bytes, void* stream) {
  clear_error();
  if (!d_count || !d_hist || !d_workspace || (k > 0 && !d_rec))
    return set_error(WEDGE_EINVAL, "wedge_triangle_stats: null pointer");
  if (!aligned(d_workspace, 256) || !aligned(d_count, 8) || !aligned(d_hist, 8) ||
      !aligned(d_rec, 4) || !aligned(d_tri, 4))
    return set_error(WEDGE_EINVAL, "wedge_triangle_stats: misaligned pointer");
  if (k >= (1ULL << 32)) return set_error(WEDGE_ERANGE, "wedge_triangle_stats: k >= 2^32");
  if (max_bins == 0 || max_bins > 64 || tau == 0 || omega < 2)
    return set_error(WEDGE_ERANGE, "wedge_triangle_stats: bad max_bins, tau or omega");
  if (workspace_bytes < wedge_triangle_stats_workspace(k))
    return set_error(WEDGE_EWORKSPACE, "wedge_triangle_stats: workspace %zu < %zu bytes",
                     workspace_bytes, wedge_triangle_stats_workspace(k));
  hipStream_t st = (hipStream_t)stream;
  int rc = fill<uint64_t>(d_hist, (uint64_t)max_bins * max_bins, 0, st);
  if (rc || (rc = fill<uint64_t>(d_count, 1, 0, st))) return rc;
  return scan_apply<uint64_t>(TriLoad{d_rec},
                              TriApply{d_rec, d_tri, d_hist, d_count, k, omega, tau, max_bins},
                              k, (uint64_t*)d_workspace, st);
}

extern "C" int wedge_triangle_box(const uint64_t* h_hist, uint32_t max_bins,
                                  wedge_triangle_box_row* h_out) {
  clear_error();
  if (!h_hist || !h_out) return set_error(WEDGE_EINVAL, "wedge_triangle_box: null pointer");
  if (max_bins == 0 || max_bins > 64)
    return set_error(WEDGE_ERANGE, "wedge_triangle_box: max_bins must be 1..64");
  for (uint32_t b = 0; b < max_bins; ++b) {
    const uint64_t* h = h_hist + (uint64_t)b * max_bins;
    wedge_triangle_box_row r{};
    for (uint32_t x = 0; x < max_bins; ++x) r.count += h[x];
    if (r.count > 0) {
      // nearest rank: smallest bin with at least ceil(p N) values at or below it
      const uint64_t N = r.count;
      const uint64_t need[3] = {(N + 3) / 4, (N + 1) / 2, (3 * N + 3) / 4};
      uint32_t q[3] = {0, 0, 0};
      for (int j = 0; j < 3; ++j) {
        uint64_t cum = 0;
        for (uint32_t x = 0; x < max_bins; ++x) {
          cum += h[x];
          if (cum >= need[j]) {
            q[j] = x;
            break;
          }
        }
      }
      r.q1 = q[0];
      r.median = q[1];
      r.q3 = q[2];
      // Tukey whiskers in half-bin units: 2x within [2 q1 - 3 IQR, 2 q3 + 3 IQR]
      const int64_t iqr = (int64_t)q[2] - (int64_t)q[0];
      const int64_t lo2 = 2 * (int64_t)q[0] - 3 * iqr, hi2 = 2 * (int64_t)q[2] + 3 * iqr;
      r.whisker_lo = q[0];
      r.whisker_hi = q[2];
      for (uint32_t x = 0; x < max_bins; ++x) {
        if (h[x] == 0) continue;
        const int64_t x2 = 2 * (int64_t)x;
        if (x2 < lo2 || x2 > hi2) {
          r.outliers += h[x];
        } else {
          if (x < r.whisker_lo) r.whisker_lo = x;
          if (x > r.whisker_hi) r.whisker_hi = x;
        }
      }
    }
    h_out[b] = r;
  }
  return WEDGE_OK;
}
