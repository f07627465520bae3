// Polynomial fitting helpers (templates), included from pswf.h.
#pragma once

#include <cmath>
#include <vector>

namespace espx {

template <class F>
std::vector<double> fit_chebyshev(F f, int deg) {
  const int n = deg + 1;
  std::vector<double> fx(n), a(n, 0.0);
  for (int j = 0; j < n; ++j) fx[j] = f(std::cos(M_PI * (j + 0.5) / n));
  for (int k = 0; k < n; ++k) {
    double s = 0;
    for (int j = 0; j < n; ++j) s += fx[j] * std::cos(M_PI * k * (j + 0.5) / n);
    a[k] = (k == 0 ? 1.0 : 2.0) * s / n;
  }
  return a;
}

template <class F>
std::vector<double> fit_monomial(F f, double a, double b, int deg) {
  const double mid = 0.5 * (a + b), half = 0.5 * (b - a);
  std::vector<double> ch = fit_chebyshev([&](double z) { return f(mid + half * z); }, deg);
  // Chebyshev -> monomials in z
  std::vector<double> mono(deg + 1, 0.0), tkm1(deg + 1, 0.0), tk(deg + 1, 0.0), tkp1(deg + 1);
  tkm1[0] = 1.0;                     // T_0
  if (deg >= 1) tk[1] = 1.0;         // T_1
  mono[0] += ch[0];
  if (deg >= 1) mono[1] += ch[1];
  for (int k = 1; k < deg; ++k) {
    for (int j = 0; j <= deg; ++j) tkp1[j] = -tkm1[j] + (j > 0 ? 2.0 * tk[j - 1] : 0.0);
    for (int j = 0; j <= deg; ++j) mono[j] += ch[k + 1] * tkp1[j];
    tkm1 = tk;
    tk = tkp1;
  }
  // monomials in z = tau / half  ->  monomials in tau
  double s = 1.0;
  for (int j = 0; j <= deg; ++j) {
    mono[j] /= s;
    s *= half;
  }
  return mono;
}

}  // namespace espx
