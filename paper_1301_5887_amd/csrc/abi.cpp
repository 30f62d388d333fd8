// Host side of libwedge: error plumbing, the binning and Hoeffding helpers,
// and the FP64 estimates of Alg. phase4c and Eq. global_est.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace wedge {

static thread_local char g_err[512] = "";

int set_error(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return status;
}

void clear_error() { g_err[0] = 0; }

}  // namespace wedge

using namespace wedge;

extern "C" const char* wedge_last_error(void) { return g_err; }

extern "C" int wedge_abi_version(void) { return 1; }

extern "C" uint64_t wedge_bin_lo_deg(uint32_t b, uint32_t tau, uint64_t omega) {
  return bin_lo_deg(b, tau, omega);
}

extern "C" uint32_t wedge_bin_id(uint64_t d, uint32_t tau, uint64_t omega) {
  // max{ b : BinLoDeg(b) <= d }; BinLoDeg is strictly increasing until it
  // saturates, so walk the bins up from tau.
  if (d <= tau) return (uint32_t)d;
  uint32_t b = tau;
  while (b < 0xFFFFFFFFu && bin_lo_deg(b + 1, tau, omega) <= d) {
    ++b;
    if (bin_lo_deg(b, tau, omega) == ~0ULL) break;
  }
  return b;
}

extern "C" uint64_t wedge_hoeffding_k(double eps, double delta) {
  if (!(eps > 0.0) || !(delta > 0.0) || !(delta < 1.0)) return 0;
  const double k = 0.5 / (eps * eps) * log(2.0 / delta);
  return (uint64_t)ceil(k);
}

extern "C" int wedge_estimate(const uint64_t* h_n_b, const uint64_t* h_p_b, const uint64_t* h_q,
                              const uint64_t* h_k, uint32_t max_bins, uint32_t tau, uint64_t omega,
                              uint64_t k_global, double delta, wedge_bin_estimate* h_bins,
                              wedge_global_estimate* h_global) {
  clear_error();
  if (!h_n_b || !h_p_b || !h_q || !h_k || !h_bins || !h_global)
    return set_error(WEDGE_EINVAL, "wedge_estimate: null pointer");
  if (!(delta > 0.0) || !(delta < 1.0))
    return set_error(WEDGE_EINVAL, "wedge_estimate: delta must be in (0, 1)");
  uint64_t p = 0;
  for (uint32_t b = 0; b < max_bins; ++b) p += h_p_b[b];
  const double lg = log(2.0 / delta);
  double num = 0.0, tsum = 0.0;
  for (uint32_t b = 0; b < max_bins; ++b) {
    wedge_bin_estimate& e = h_bins[b];
    const uint64_t* q = h_q + (uint64_t)b * 4;
    e.bin = b;
    e.lo_deg = bin_lo_deg(b, tau, omega);
    e.n_b = h_n_b[b];
    e.p_b = h_p_b[b];
    e.k_b = h_k[b];
    for (int i = 0; i < 4; ++i) e.q[i] = q[i];
    e.valid = h_k[b] > 0;
    e.c = e.t = e.eps = 0.0;
    if (e.valid) {
      const double k = (double)h_k[b];
      e.c = (double)(q[1] + q[2] + q[3]) / k;
      const uint64_t t6 = 6 * q[1] + 3 * q[2] + 2 * q[3];
      e.t = ((double)h_p_b[b] * (double)t6) / (6.0 * k);
      e.eps = sqrt(lg / (2.0 * k));
    }
    num += (double)h_p_b[b] * e.c;
    tsum += e.t;
  }
  const uint64_t* qg = h_q + (uint64_t)max_bins * 4;
  h_global->p = p;
  h_global->k_global = k_global;
  for (int i = 0; i < 4; ++i) h_global->q_global[i] = qg[i];
  h_global->c = p > 0 ? num / (double)p : 0.0;
  h_global->t = h_global->c * (double)p / 3.0;
  h_global->c_global = k_global > 0 ? (double)qg[3] / (double)k_global : 0.0;
  h_global->t_global = h_global->c_global * (double)p / 3.0;
  h_global->eps_global = k_global > 0 ? sqrt(lg / (2.0 * (double)k_global)) : 0.0;
  h_global->t_bins_sum = tsum;
  return WEDGE_OK;
}
