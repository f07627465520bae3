// FP64 host numerics of psi_0^c; see pswf.h.
#include "pswf.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace espx {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(z), p0 = P_{n-1}(z)
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal (a, b) below s.
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double s) {
  int cnt = 0;
  double d = a[0] - s;
  if (d < 0) ++cnt;
  for (size_t i = 1; i < a.size(); ++i) {
    if (d == 0.0) d = 1e-300;
    d = a[i] - s - b[i - 1] * b[i - 1] / d;
    if (d < 0) ++cnt;
  }
  return cnt;
}

}  // namespace

Pswf::Pswf(double c) : c_(c) {
  if (!(c > 0.0)) throw std::invalid_argument("PSWF bandwidth must be positive");
  const int K = static_cast<int>(1.5 * c) + 40;
  std::vector<double> a(K), b(K - 1);
  for (int k = 0; k < K; ++k) {
    const double n = 2.0 * k;
    a[k] = n * (n + 1) + c * c * (2 * n * (n + 1) - 1) / ((2 * n + 3) * (2 * n - 1));
    if (k + 1 < K)
      b[k] = c * c * (n + 2) * (n + 1) / ((2 * n + 3) * std::sqrt((2 * n + 1) * (2 * n + 5)));
  }
  // smallest eigenvalue by bisection on the Sturm count
  double lo = a[0], hi = a[0];
  for (int k = 0; k < K; ++k) {
    double r = (k > 0 ? std::fabs(b[k - 1]) : 0.0) + (k + 1 < K ? std::fabs(b[k]) : 0.0);
    lo = std::min(lo, a[k] - r);
  }
  for (int it = 0; it < 400 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(a, b, mid) >= 1) hi = mid; else lo = mid;
  }
  const double lam = lo - 1e-11 * std::max(1.0, std::fabs(lo));
  // inverse iteration with the LDL^T (Thomas) solver of T - lam I
  std::vector<double> v(K, 1.0), d(K), l(K), y(K);
  for (int it = 0; it < 4; ++it) {
    d[0] = a[0] - lam;
    for (int k = 1; k < K; ++k) {
      l[k] = b[k - 1] / d[k - 1];
      d[k] = a[k] - lam - l[k] * b[k - 1];
    }
    y[0] = v[0];
    for (int k = 1; k < K; ++k) y[k] = v[k] - l[k] * y[k - 1];
    v[K - 1] = y[K - 1] / d[K - 1];
    for (int k = K - 2; k >= 0; --k) v[k] = (y[k] - b[k] * v[k + 1]) / d[k];
    double nrm = 0;
    for (double e : v) nrm += e * e;
    nrm = std::sqrt(nrm);
    for (double& e : v) e /= nrm;
  }
  // coefficients of the standard P_{2k}: Pbar_n = sqrt(n + 1/2) P_n
  a_.resize(K);
  for (int k = 0; k < K; ++k) a_[k] = v[k] * std::sqrt(2.0 * k + 0.5);
  double d0;
  if (series(0.0, &d0) < 0)
    for (double& e : a_) e = -e;
  psi0_ = series(0.0, &d0);
  C0_ = a_[0];                       // int_0^1 P_0 = 1, int_0^1 P_{2k} = 0 for k >= 1
  lam0_ = 2.0 * C0_ / psi0_;         // eq. psidefinit at x = 0
  gauss_legendre(static_cast<int>(2 * c) + 80, qt_, qw_);
  qpsi_.resize(qt_.size());
  for (size_t j = 0; j < qt_.size(); ++j) qpsi_[j] = series(qt_[j], &d0);
}

double Pswf::series(double x, double* deriv) const {
  // P_n and P'_n by the three-term recurrences; only even n contribute
  double p0 = 1.0, p1 = x, dp0 = 0.0, dp1 = 1.0;
  double s = a_[0], ds = 0.0;
  const int nmax = 2 * static_cast<int>(a_.size()) - 2;
  for (int n = 1; n < nmax; ++n) {
    double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
    double dp2 = (n + 1.0) * p1 + x * dp1;
    p0 = p1; p1 = p2;
    dp0 = dp1; dp1 = dp2;
    if ((n + 1) % 2 == 0) {
      s += a_[(n + 1) / 2] * p1;
      ds += a_[(n + 1) / 2] * dp1;
    }
  }
  (void)dp0;
  *deriv = ds;
  return s;
}

double Pswf::psi(double x) const {
  if (std::fabs(x) <= 1.0) {
    double d;
    return series(x, &d);
  }
  double s = 0;
  for (size_t j = 0; j < qt_.size(); ++j) s += qw_[j] * qpsi_[j] * std::cos(c_ * x * qt_[j]);
  return s / lam0_;
}

double Pswf::dpsi(double x) const {
  if (std::fabs(x) <= 1.0) {
    double d;
    series(x, &d);
    return d;
  }
  double s = 0;
  for (size_t j = 0; j < qt_.size(); ++j)
    s -= qw_[j] * qpsi_[j] * c_ * qt_[j] * std::sin(c_ * x * qt_[j]);
  return s / lam0_;
}

double Pswf::int_psi(double x) const {
  // int_0^x P_0 = x; int_0^x P_n = (P_{n+1} - P_{n-1}) / (2n + 1) for even n >= 2
  const int nmax = 2 * static_cast<int>(a_.size());
  std::vector<double> P(nmax + 1);
  P[0] = 1.0;
  P[1] = x;
  for (int n = 1; n < nmax; ++n) P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
  double s = a_[0] * x;
  for (size_t k = 1; k < a_.size(); ++k) {
    const int n = 2 * static_cast<int>(k);
    s += a_[k] * (P[n + 1] - P[n - 1]) / (2.0 * n + 1.0);
  }
  return s;
}

double c_from_delta(double delta) {
  if (!(delta >= 1e-14 && delta < 1.0)) throw std::invalid_argument("Delta out of range");
  auto g = [&](double c) {
    Pswf p(c);
    return std::log(p.psi(1.0) / p.psi0()) - std::log(delta);
  };
  double lo = 0.05, hi = 36.0;
  double glo = g(lo);
  for (int it = 0; it < 80 && hi - lo > 1e-13; ++it) {
    double mid = 0.5 * (lo + hi);
    double gm = g(mid);
    if ((gm > 0) == (glo > 0)) { lo = mid; glo = gm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

}  // namespace espx
