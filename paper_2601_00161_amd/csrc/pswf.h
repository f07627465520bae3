// Host-side FP64 numerics of the order-zero prolate spheroidal wave function
// psi_0^c and the polynomial tables the device kernels evaluate.
//
// psi_0^c is the eigenfunction of the largest eigenvalue of the operator
// phi -> int_{-1}^{1} phi(t) exp(i c x t) dt (paper, App. A.1, eq. psidefinit),
// normalised to unit L2 norm.  It is computed as the ground state of the
// commuting prolate differential operator -((1-x^2) psi')' + c^2 x^2 psi in a
// normalised even-Legendre basis (a symmetric tridiagonal matrix: bisection
// on Sturm counts for the eigenvalue, then inverse iteration).
#pragma once

#include <vector>

namespace espx {

class Pswf {
 public:
  explicit Pswf(double c);
  double c() const { return c_; }
  // psi(x); |x| <= 1 from the Legendre series, beyond from the eigen-equation
  // (1/lam0) int_{-1}^{1} psi(t) cos(c x t) dt, which is also the exact
  // Fourier transform of the window continued past its band.
  double psi(double x) const;
  double dpsi(double x) const;          // derivative, any x
  double int_psi(double x) const;       // int_0^x psi, |x| <= 1
  double psi0() const { return psi0_; }
  double C0() const { return C0_; }     // int_0^1 psi
  double lambda0() const { return lam0_; }  // = 2 C0 / psi(0) (eq. psidefinit at x = 0)

 private:
  double series(double x, double* deriv) const;
  double c_;
  std::vector<double> a_;   // coefficients of P_{2k} (standard Legendre) for k = 0..K-1
  std::vector<double> qt_, qw_, qpsi_;  // Gauss-Legendre nodes, weights, psi at nodes
  double psi0_ = 0, C0_ = 0, lam0_ = 0;
};

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Bandwidth c with psi_0^c(1) / psi_0^c(0) = delta (parameter rule of Sec. 5.1).
double c_from_delta(double delta);

// Monomial coefficients (in tau) of the Chebyshev interpolant of degree deg of
// f on [a, b], expressed around the interval centre: f(mid + tau) ~ sum_j c_j tau^j.
template <class F>
std::vector<double> fit_monomial(F f, double a, double b, int deg);

// Chebyshev coefficients of the degree-deg interpolant of f on [-1, 1].
template <class F>
std::vector<double> fit_chebyshev(F f, int deg);

}  // namespace espx

#include "pswf_fit.inl"
