// Host side of the learned control variate: the estimator arithmetic.
//
// The closed fraction c_b of a bin (Thm. cd-est) is estimated from EVAL
// draws X (exact closure labels) and the network's g by
//     c_CV = mean(X - beta g) + beta mu,
// with beta fixed from held-out TRAIN draws before any EVAL draw and mu the
// mean of g over the bin's wedges: exact (from the census), or the mean of
// an independent second sample (AUX draws of g, or centre draws of gbar).
// Draws come in rounds; after round i the two-sided empirical-Bernstein
// half-width (Maurer & Pontil 2009, Thm. 4) at delta_i = delta / (i (i+1))
// (a union bound over rounds) decides whether the row needs more draws.
// Every input is an integer moment sum of wedge_cv_moments (terms rounded to
// 2^-32, so the sums do not depend on the order of the draws); this file
// turns them into beta, variances, estimates, half-widths, stop decisions
// and round plans, and sequences the training draws (wedge_cv_train).
#include <math.h>
#include <string.h>

#include <vector>

#include "common.hpp"
#include "scan.hpp"

namespace wedge {

namespace {

constexpr double kQ32 = 4294967296.0;  // 2^32: scale of the g sums

// Empirical-Bernstein half-width of the mean of n values in an interval of
// length R with sample variance var (n - 1 denominator), two-sided with
// delta/2 per side; +inf for n < 2.
double eb_halfwidth(uint64_t n, double var, double R, double delta) {
  if (n < 2) return INFINITY;
  if (var < 0.0) var = 0.0;
  const double L = log(4.0 / delta);
  return sqrt(2.0 * var * L / (double)n) + 7.0 * R * L / (3.0 * (double)(n - 1));
}

// Smallest planning n with eb_halfwidth(n, var, R, delta) <= eps when n - 1 is
// taken as n (then one draw added): the positive root x = 1/sqrt(n) of
// a x + b x^2 = eps with a = sqrt(2 var ln(4/delta)), b = 7 R ln(4/delta) / 3.
double eb_samples(double var, double R, double delta, double eps) {
  const double L = log(4.0 / delta);
  const double a = sqrt(2.0 * (var > 0.0 ? var : 0.0) * L);
  const double b = 7.0 * R * L / 3.0;
  const double x = 2.0 * eps / (a + sqrt(a * a + 4.0 * b * eps));
  return ceil(1.0 / (x * x)) + 1.0;
}

struct Moments {
  double n, mx, mg, vx, vg, cxg;
};

// Means and (n - 1)-denominator variances and covariance from the integer
// moments [count, sum X, 2^32 sum g, 2^32 sum g^2, 2^32 sum X g].
Moments moments_of(int64_t n, int64_t sx, int64_t sg, int64_t sg2, int64_t sxg) {
  Moments M;
  M.n = (double)n;
  M.mx = (double)sx / M.n;
  M.mg = (double)sg / kQ32 / M.n;
  M.vx = ((double)sx - M.n * M.mx * M.mx) / (M.n - 1.0);
  M.vg = ((double)sg2 / kQ32 - M.n * M.mg * M.mg) / (M.n - 1.0);
  M.cxg = ((double)sxg / kQ32 - M.n * M.mx * M.mg) / (M.n - 1.0);
  return M;
}

}  // namespace

}  // namespace wedge

using namespace wedge;

extern "C" double wedge_eb_halfwidth(uint64_t n, double var, double R, double delta) {
  return wedge::eb_halfwidth(n, var, R, delta);
}

extern "C" uint64_t wedge_eb_samples(double var, double R, double delta, double eps) {
  if (!(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0) || !(R > 0.0)) return 0;
  return (uint64_t)wedge::eb_samples(var, R, delta, eps);
}

extern "C" uint64_t wedge_cv_round_size(uint64_t first, double growth, uint32_t round,
                                        uint64_t max_per_row) {
  if (round == 0) return 0;
  const double t = ceil((double)first * pow(growth, (double)(round - 1)));
  return t >= (double)max_per_row ? max_per_row : (uint64_t)t;
}

extern "C" int wedge_cv_fit(const int64_t* h_mom, uint32_t rows, double eps, double delta,
                            wedge_cv_fit_row* h_out) {
  clear_error();
  if (!h_mom || !h_out) return set_error(WEDGE_EINVAL, "wedge_cv_fit: null pointer");
  if (!(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0))
    return set_error(WEDGE_EINVAL, "wedge_cv_fit: eps > 0 and 0 < delta < 1 required");
  for (uint32_t r = 0; r < rows; ++r) {
    const int64_t* m = h_mom + 5 * (uint64_t)r;
    wedge_cv_fit_row& o = h_out[r];
    o.beta = o.rho2 = 0.0;
    o.var_x = o.var_z = 0.25;
    if (m[0] >= 2) {
      // beta and rho^2 from the population (n-denominator) moments: the
      // least-squares coefficient of X on g and the squared correlation
      const double n = (double)m[0];
      const double mx = (double)m[1] / n, mg = (double)m[2] / kQ32 / n;
      const double cov = (double)m[4] / kQ32 / n - mx * mg;
      const double vg = (double)m[3] / kQ32 / n - mg * mg;
      const double vx = mx - mx * mx;
      if (vg > 1e-14) o.beta = cov / vg;
      if (vx > 0.0 && vg > 1e-14) o.rho2 = cov * cov / (vx * vg);
      const Moments M = moments_of(m[0], m[1], m[2], m[3], m[4]);
      o.var_x = M.vx;
      const double vz = M.vx - 2.0 * o.beta * M.cxg + o.beta * o.beta * M.vg;
      o.var_z = vz > 0.0 ? vz : 0.0;
    }
    // first-round sizes at delta / 2 (the first round's share of the union
    // bound): plain (range 1) and control variate (range 1 + |beta|)
    o.plan_plain = (uint64_t)eb_samples(o.var_x, 1.0, delta / 2.0, eps);
    o.plan_cv = (uint64_t)eb_samples(o.var_z, 1.0 + fabs(o.beta), delta / 2.0, eps);
  }
  return WEDGE_OK;
}

extern "C" int wedge_cv_estimate(const wedge_cv_row* h_rows, uint32_t nrows, uint32_t round,
                                 double delta, double eps, uint64_t max_per_row,
                                 wedge_cv_result* h_out) {
  clear_error();
  if (!h_rows || !h_out) return set_error(WEDGE_EINVAL, "wedge_cv_estimate: null pointer");
  if (round == 0 || !(delta > 0.0) || !(delta < 1.0) || !(eps > 0.0))
    return set_error(WEDGE_EINVAL, "wedge_cv_estimate: round >= 1, eps > 0, 0 < delta < 1");
  for (uint32_t r = 0; r < nrows; ++r)
    if (h_rows[r].mode > WEDGE_CV_CENTRE)
      return set_error(WEDGE_EINVAL, "wedge_cv_estimate: row %u has mode %u", r, h_rows[r].mode);
  const double di = delta / ((double)round * ((double)round + 1.0));
  for (uint32_t r = 0; r < nrows; ++r) {
    const wedge_cv_row& s = h_rows[r];
    wedge_cv_result& o = h_out[r];
    o.estimate = NAN;
    o.halfwidth = INFINITY;
    if (s.n >= 2) {
      const Moments M = moments_of(s.n, s.sx, s.sg, s.sg2, s.sxg);
      const double b = s.beta;
      const double vz = M.vx - 2.0 * b * M.cxg + b * b * M.vg;
      const double R = 1.0 + fabs(b);
      if (s.mode == WEDGE_CV_PLAIN || (s.mode == WEDGE_CV_CENTRE && b == 0.0)) {
        o.estimate = M.mx;
        o.halfwidth = eb_halfwidth(s.n, M.vx, 1.0, di);
      } else if (s.mode == WEDGE_CV_EXACT) {
        o.estimate = (M.mx - b * M.mg) + b * s.exact_mean;
        o.halfwidth = eb_halfwidth(s.n, vz, R, di);
      } else if (s.an >= 2) {
        // the second sample (AUX g, or centre gbar) estimates mu; each side
        // of the bound takes delta_i / 2
        const double an = (double)s.an;
        const double am = (double)s.ag / kQ32 / an;
        const double av = ((double)s.ag2 / kQ32 - an * am * am) / (an - 1.0);
        o.estimate = (M.mx - b * M.mg) + b * am;
        o.halfwidth = eb_halfwidth(s.n, vz, R, di / 2.0) +
                      fabs(b) * eb_halfwidth(s.an, av, 1.0, di / 2.0);
      }
    }
    o.more = (o.halfwidth > eps && s.done < max_per_row) ? 1 : 0;
  }
  return WEDGE_OK;
}

extern "C" int wedge_cv_bin_means(const double* h_key_sum, const uint64_t* h_key_count,
                                  const uint32_t* h_key_bin, uint32_t nkeys, uint32_t max_bins,
                                  double* h_mean, uint64_t* h_count) {
  clear_error();
  if (!h_key_sum || !h_key_count || !h_key_bin || !h_mean || !h_count)
    return set_error(WEDGE_EINVAL, "wedge_cv_bin_means: null pointer");
  for (uint32_t b = 0; b <= max_bins; ++b) {
    h_mean[b] = 0.0;
    h_count[b] = 0;
  }
  // sums per bin in key order (keys run in increasing degree order)
  for (uint32_t k = 0; k < nkeys; ++k) {
    const uint32_t b = h_key_bin[k];
    if (b >= max_bins) return set_error(WEDGE_EINVAL, "wedge_cv_bin_means: key %u bin %u", k, b);
    h_mean[b] += h_key_sum[k];
    h_count[b] += h_key_count[k];
  }
  double num = 0.0;
  uint64_t den = 0;
  for (uint32_t b = 0; b < max_bins; ++b) {
    num += h_mean[b];
    den += h_count[b];
    h_mean[b] = h_count[b] > 0 ? h_mean[b] / (double)h_count[b] : 0.0;
  }
  h_mean[max_bins] = den > 0 ? num / (double)den : 0.0;
  h_count[max_bins] = den;
  return WEDGE_OK;
}

extern "C" int wedge_cv_mean_var(const int64_t* h_mom, uint32_t rows, double* h_mean,
                                 double* h_var) {
  clear_error();
  if (!h_mom || !h_mean || !h_var) return set_error(WEDGE_EINVAL, "wedge_cv_mean_var: null");
  for (uint32_t r = 0; r < rows; ++r) {
    const int64_t* m = h_mom + 5 * (uint64_t)r;
    h_mean[r] = NAN;
    h_var[r] = 0.0;
    if (m[0] < 1) continue;
    const double n = (double)m[0];
    const double mean = (double)m[2] / kQ32 / n;
    h_mean[r] = mean;
    if (m[0] >= 2) {
      const double v = ((double)m[3] / kQ32 - n * mean * mean) / (n - 1.0);
      h_var[r] = v > 0.0 ? v : 0.0;
    }
  }
  return WEDGE_OK;
}

extern "C" double wedge_cv_centre_cost(const uint64_t* h_n_b, const uint64_t* h_p_b,
                                       uint32_t max_bins, uint32_t row, double a, double b) {
  // degree d of a typical centre of row r: the d whose C(d, 2) is the row's
  // mean wedges per vertex; the global row weights the bins by their wedges
  auto deg = [&](uint32_t k) {
    const double nb = (double)h_n_b[k], pb = (double)h_p_b[k];
    return nb > 0.0 ? 0.5 + sqrt(0.25 + 2.0 * pb / nb) : 0.0;
  };
  double d;
  if (row < max_bins) {
    d = deg(row);
  } else {
    double num = 0.0, den = 0.0;
    for (uint32_t k = 0; k < max_bins; ++k) {
      if (h_p_b[k] == 0) continue;
      num += (double)h_p_b[k] * deg(k);
      den += (double)h_p_b[k];
    }
    d = num / (den > 1.0 ? den : 1.0);
  }
  return 1.0 + a * pow(d, b);
}

extern "C" int wedge_cv_plan_centre(const wedge_cv_fit_row* h_fit, const double* h_centre_var,
                                    const double* h_cost, uint32_t rows, double eps, double delta,
                                    uint64_t* h_eval, uint64_t* h_centre, double* h_beta) {
  clear_error();
  if (!h_fit || !h_centre_var || !h_cost || !h_eval || !h_centre || !h_beta)
    return set_error(WEDGE_EINVAL, "wedge_cv_plan_centre: null pointer");
  if (!(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0))
    return set_error(WEDGE_EINVAL, "wedge_cv_plan_centre: eps > 0 and 0 < delta < 1 required");
  for (uint32_t r = 0; r < rows; ++r) {
    const wedge_cv_fit_row& f = h_fit[r];
    const double plain = eb_samples(f.var_x, 1.0, delta / 2.0, eps);
    h_eval[r] = (uint64_t)plain;
    h_centre[r] = 0;
    h_beta[r] = 0.0;
    if (f.beta == 0.0) continue;
    // share t of eps for the centre term, on a grid of 0.01 .. 0.99; each
    // term of the bound at delta / 4 (first round's delta / 2, split in two)
    const double ab = fabs(f.beta);
    double best = INFINITY, bne = 0.0, bnc = 0.0;
    for (int i = 1; i < 100; ++i) {
      const double t = 0.01 * i;
      const double ne = eb_samples(f.var_z, 1.0 + ab, delta / 4.0, eps * (1.0 - t));
      const double nc = eb_samples(h_centre_var[r], 1.0, delta / 4.0, eps * t / ab);
      const double cost = ne + h_cost[r] * nc;
      if (cost < best) {
        best = cost;
        bne = ne;
        bnc = nc;
      }
    }
    if (best < plain) {
      h_eval[r] = (uint64_t)bne;
      h_centre[r] = (uint64_t)bnc;
      h_beta[r] = f.beta;
    }
  }
  return WEDGE_OK;
}

// ------------------------------------------------------------ training draws
namespace {

struct TrainLayout {
  size_t fit, hold, g, mom, loss, train, total;
};

TrainLayout train_layout(uint32_t rows, uint64_t n_fit, uint64_t n_hold, uint64_t batch) {
  TrainLayout L;
  size_t off = 0;
  L.fit = off;
  off += round_up((size_t)rows * n_fit * sizeof(wedge_feature_rec) + 1, 256);
  L.hold = off;
  off += round_up((size_t)rows * n_hold * sizeof(wedge_feature_rec) + 1, 256);
  L.g = off;
  off += round_up((size_t)rows * n_hold * sizeof(float) + 1, 256);
  L.mom = off;
  off += round_up((size_t)rows * 5 * sizeof(int64_t), 256);
  L.loss = off;
  off += 256;
  L.train = off;
  off += round_up(wedge_mlp_train_workspace(rows, batch), 256);
  L.total = off;
  return L;
}

}  // namespace

extern "C" size_t wedge_cv_train_workspace(uint32_t rows, uint64_t n_fit, uint64_t n_hold,
                                           uint64_t per_row_batch) {
  return train_layout(rows, n_fit, n_hold, per_row_batch).total;
}

extern "C" int wedge_cv_train(const uint64_t* d_rowptr, const uint32_t* d_col, uint32_t n,
                              uint64_t m, const void* d_index, uint32_t max_bins, uint32_t tau,
                              uint64_t omega, const uint32_t* h_rows, uint32_t nrows,
                              uint64_t n_fit, uint64_t n_hold, uint64_t per_row_batch,
                              uint32_t epochs, float lr, uint64_t seed, uint64_t init_seed,
                              void* d_state, double eps, double delta, wedge_cv_fit_row* h_fit,
                              int64_t* h_mom, float* h_loss, void* d_workspace,
                              size_t workspace_bytes, void* stream) {
  clear_error();
  if (!h_rows || !h_fit || !d_state || !d_workspace)
    return set_error(WEDGE_EINVAL, "wedge_cv_train: null pointer");
  if (nrows == 0 || n_fit == 0 || n_hold < 2 || per_row_batch == 0 || n_fit % per_row_batch)
    return set_error(WEDGE_EINVAL,
                     "wedge_cv_train: rows >= 1, n_hold >= 2 and n_fit a positive multiple of "
                     "per_row_batch required");
  if (!aligned(d_workspace, 256)) return set_error(WEDGE_EINVAL, "wedge_cv_train: misaligned");
  for (uint32_t j = 0; j < nrows; ++j)
    if (h_rows[j] > max_bins || (j > 0 && h_rows[j] <= h_rows[j - 1]))
      return set_error(WEDGE_EINVAL, "wedge_cv_train: rows must be increasing and <= max_bins");
  const TrainLayout L = train_layout(nrows, n_fit, n_hold, per_row_batch);
  if (workspace_bytes < L.total)
    return set_error(WEDGE_EWORKSPACE, "wedge_cv_train: workspace %zu < %zu bytes",
                     workspace_bytes, L.total);
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)d_workspace;
  wedge_feature_rec* fit = (wedge_feature_rec*)(w + L.fit);
  wedge_feature_rec* hold = (wedge_feature_rec*)(w + L.hold);
  float* g = (float*)(w + L.g);
  int64_t* mom = (int64_t*)(w + L.mom);
  float* loss = (float*)(w + L.loss);
  // TRAIN draws 0 .. n_fit - 1 of every row fit the network; n_fit ..
  // n_fit + n_hold - 1 are held out for beta, rho^2 and the round plans
  uint64_t hk[4097], sb[4097];
  if (max_bins > 4096) return set_error(WEDGE_ERANGE, "wedge_cv_train: max_bins > 4096");
  memset(hk, 0, sizeof(uint64_t) * (max_bins + 1));
  memset(sb, 0, sizeof(uint64_t) * (max_bins + 1));
  for (uint32_t j = 0; j < nrows; ++j) hk[h_rows[j]] = n_fit;
  int rc = wedge_sample_features(d_rowptr, d_col, n, m, d_index, max_bins, tau, omega, hk, sb,
                                 seed, WEDGE_DOMAIN_TRAIN, 0, 1, fit, n_fit, nullptr, stream);
  if (rc) return rc;
  for (uint32_t j = 0; j < nrows; ++j) {
    hk[h_rows[j]] = n_hold;
    sb[h_rows[j]] = n_fit;
  }
  rc = wedge_sample_features(d_rowptr, d_col, n, m, d_index, max_bins, tau, omega, hk, sb, seed,
                             WEDGE_DOMAIN_TRAIN, 0, 1, hold, n_hold, nullptr, stream);
  if (rc) return rc;
  if ((rc = wedge_mlp_init(d_state, init_seed, stream))) return rc;
  if ((rc = wedge_mlp_train(d_state, fit, nrows, n_fit, n_fit, per_row_batch, epochs, 0, lr, 0.9f,
                            0.999f, 1e-8f, loss, w + L.train, workspace_bytes - L.train, stream)))
    return rc;
  if ((rc = wedge_mlp_forward(d_state, hold, (uint64_t)nrows * n_hold, g, stream))) return rc;
  if ((rc = fill<int64_t>(mom, (uint64_t)nrows * 5, 0, st))) return rc;
  if ((rc = wedge_cv_moments(hold, g, nrows, n_hold, n_hold, nullptr, mom, stream))) return rc;
  std::vector<int64_t> hm((size_t)nrows * 5);
  float hl = 0.0f;
  // both copies land in host memory of this frame, so the stream is drained
  // before any return
  hipError_t e = hipMemcpyAsync(hm.data(), mom, hm.size() * sizeof(int64_t),
                                hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&hl, loss, sizeof(float), hipMemcpyDeviceToHost, st);
  const hipError_t es = hipStreamSynchronize(st);
  WEDGE_HIP_TRY(e);
  WEDGE_HIP_TRY(es);
  if (h_mom) memcpy(h_mom, hm.data(), hm.size() * sizeof(int64_t));
  if (h_loss) *h_loss = hl;
  return wedge_cv_fit(hm.data(), nrows, eps, delta, h_fit);
}
