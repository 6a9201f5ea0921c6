// Host-only parameter selection of libqsw: theta_m from its definition and
// the Taylor degree / scaling choice.  Compiled as plain C++ (no device code).
#include "params.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace qsw {

namespace {

constexpr int kMMax = 55;  // largest Taylor degree
constexpr int kPMax = 8;   // largest p in alpha_p = max(d_p, d_{p+1})
// Single-precision products: the degree is capped so that the terms of a
// scaling step stay within e^theta_20 (about 35) of its input; p_max is then
// the largest p with p(p-1)-1 <= 20.
constexpr int kMMax32 = 20;
constexpr int kPMax32 = 5;
constexpr int kEll = 2;    // columns of the block 1-norm estimator

// ---------------------------------------------------------------- theta_m
//
// theta_m = max{theta : sum_{k>m} |c_k| theta^(k-1) <= tol} where
// h_{m+1}(x) = log(exp(-x) T_m(x)) = sum_{k>m} c_k x^k is the backward-error
// function of the truncated Taylor method (Section 3.1).  The coefficients
// g_k of log T_m satisfy T_m g' = T_m'; since log T_m agrees with x up to
// degree m, g_1 = 1, g_2..g_m = 0, and for k > m (where T_m has no x^k term)
//     k g_k = -sum_{i=k-m}^{k-1} i g_i / (k-i)!.
// The recurrence cancels heavily (about 20 digits near k = 2m), so it runs
// in binary128; the series is summed to k = m + 600, far past convergence.
typedef __float128 quad;

constexpr int kSeriesExtra = 600;

quad qabs(quad x) { return x < 0 ? -x : x; }

struct ThetaTable {
  double th[kMMax + 1];
};

void compute_theta(quad tol, ThetaTable &T) {
  T.th[0] = 0.0;
  for (int m = 1; m <= kMMax; ++m) {
    const int K = m + kSeriesExtra;
    std::vector<quad> inv_fact(m + 1);
    inv_fact[0] = 1;
    for (int i = 1; i <= m; ++i) inv_fact[i] = inv_fact[i - 1] / (quad)i;
    std::vector<quad> g(K + 1, (quad)0);
    g[1] = 1;
    for (int k = m + 1; k <= K; ++k) {
      quad acc = 0;
      for (int i = std::max(1, k - m); i <= k - 1; ++i) acc += (quad)i * g[i] * inv_fact[k - i];
      g[k] = -acc / (quad)k;
    }
    std::vector<quad> a(K + 1);
    for (int k = m + 1; k <= K; ++k) a[k] = qabs(g[k]);
    auto ratio = [&](double theta) {
      const quad th = theta;
      quad s = 0;
      for (int k = K; k >= m + 1; --k) s = s * th + a[k];
      quad p = 1;
      for (int i = 0; i < m; ++i) p *= th;
      return s * p;  // sum_{k=m+1}^{K} |c_k| theta^(k-1)
    };
    double lo = 0.0, hi = 1.0;
    while (ratio(hi) <= tol) {
      lo = hi;
      hi *= 2.0;
    }
    for (int it = 0; it < 400; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (mid == lo || mid == hi) break;
      if (ratio(mid) <= tol) lo = mid;
      else hi = mid;
    }
    T.th[m] = lo;
  }
}

const ThetaTable &table(int prec) {
  static ThetaTable tables[2];
  static std::once_flag once[2];
  const int i = prec == QSW_PREC_DOUBLE ? 0 : 1;
  std::call_once(once[i], [i] {
    quad tol = 1;
    for (int k = 0; k < (i == 1 ? 24 : 53); ++k) tol /= 2;
    compute_theta(tol, tables[i]);
  });
  return tables[i];
}

}  // namespace

double theta_of(int m, int prec) { return table(prec).th[m]; }

double tol_of(int prec) {
  return prec == QSW_PREC_DOUBLE ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
}

int mmax_of(int prec) { return prec == QSW_PREC_FP32 ? kMMax32 : kMMax; }

// Al-Mohy and Higham's choice (cited in Section 3.1): when ||tL||_1 is at
// most 2 ell p_max (p_max + 3) theta_{m_max} / (n0 m_max) the 1-norm alone
// decides, m* = argmin m ceil(||tL||_1 / theta_m); otherwise
// m * ceil(alpha_p / theta_m) is minimised over 2 <= p <= p_max and
// p(p-1)-1 <= m <= m_max with alpha_p = t max(d_p, d_{p+1}).  Ties go to the
// smallest m; s = max(1, ceil(.)).  The switch weighs the products spent on
// estimating the d_p against those they save; with `switch313` false the
// alpha_p rule decides whenever d is given (the d_p already estimated).
qsw_status_t select_params_impl(double norm1, const double *d, double t, int n0, int prec,
                                int *m_out, int *s_out, bool switch313) {
  if (!m_out || !s_out || n0 < 1 || !(norm1 >= 0.0) || !std::isfinite(t)) return QSW_ERR_ARG;
  const ThetaTable &T = table(prec);
  const int mmax = mmax_of(prec), pmax = prec == QSW_PREC_FP32 ? kPMax32 : kPMax;
  t = std::fabs(t);
  const double x = t * norm1;
  if (!std::isfinite(x)) return QSW_ERR_NONFINITE;
  if (x == 0.0) {
    *m_out = 0;
    *s_out = 1;
    return QSW_OK;
  }
  const double bound =
      2.0 * kEll * pmax * (pmax + 3) * T.th[mmax] / ((double)n0 * (double)mmax);
  int best_m = -1;
  double best_cost = 0.0, best_s = 0.0;
  if (d == nullptr || (switch313 && x <= bound)) {
    for (int m = 1; m <= mmax; ++m) {
      const double sm = std::ceil(x / T.th[m]);
      const double cost = m * sm;
      if (best_m < 0 || cost < best_cost) {
        best_m = m;
        best_cost = cost;
        best_s = sm;
      }
    }
  } else {
    for (int p = 2; p <= pmax + 1; ++p)
      if (!(d[p] >= 0.0) || !std::isfinite(d[p])) return QSW_ERR_ARG;
    for (int m = 1; m <= mmax; ++m) {
      double sm = -1.0;
      for (int p = 2; p <= pmax; ++p) {
        if (p * (p - 1) - 1 > m) break;
        const double alpha = t * std::max(d[p], d[p + 1]);
        const double sp = std::ceil(alpha / T.th[m]);
        if (sm < 0.0 || sp < sm) sm = sp;
      }
      if (sm < 0.0) continue;
      const double cost = m * sm;
      if (best_m < 0 || cost < best_cost) {
        best_m = m;
        best_cost = cost;
        best_s = sm;
      }
    }
  }
  if (best_s < 1.0) best_s = 1.0;
  if (best_s > 1.0e9) return QSW_ERR_ARG;  // t ||L|| absurdly large
  *m_out = best_m;
  *s_out = (int)best_s;
  return QSW_OK;
}

}  // namespace qsw

extern "C" {

double qsw_theta(int32_t m, int32_t prec) {
  if (m < 1 || m > qsw::kMMax ||
      (prec != QSW_PREC_DOUBLE && prec != QSW_PREC_SINGLE && prec != QSW_PREC_FP32))
    return -1.0;
  return qsw::theta_of(m, prec);
}

qsw_status_t qsw_select_params(double norm1, const double *d, double t, int32_t n0, int32_t prec,
                               int32_t *m, int32_t *s) {
  const bool known = (prec & QSW_PARAMS_KNOWN_NORMS) != 0;
  prec &= ~QSW_PARAMS_KNOWN_NORMS;
  if (prec != QSW_PREC_DOUBLE && prec != QSW_PREC_SINGLE && prec != QSW_PREC_FP32)
    return QSW_ERR_ARG;
  int mm = 0, ss = 0;
  qsw_status_t st = qsw::select_params_impl(norm1, d, t, n0, prec, &mm, &ss, !known);
  if (st == QSW_OK) {
    *m = mm;
    *s = ss;
  }
  return st;
}

}  // extern "C"
