"""Pins of the oracle's prolate spheroidal wave function (paper, App. A.1).

psi_0^c is checked against the paper's defining integral eigen-equation
(eq. psidefinit), against SciPy's independent prolate routines, and against
the consequences the paper draws from it (lam0 = 2 C0 / psi(0) at x = 0).
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import pro_ang1, pro_rad1

from oracle.pswf import PSWF, c_from_tol

CS = [2.0, 9.26, 11.68, 14.08, 20.0, 30.0]


@pytest.mark.parametrize("c", CS)
def test_eigen_equation_residual(c):
    """lam0 psi(x) = int_{-1}^{1} psi(t) cos(c x t) dt (eq. psidefinit, even part)."""
    p = PSWF(c)
    x = np.linspace(-1.0, 1.0, 23)
    rhs = np.array([integrate.quad(lambda t: float(p.psi(t)) * np.cos(c * xi * t), -1, 1,
                                   epsabs=1e-15, epsrel=1e-13, limit=200)[0] for xi in x])
    assert np.max(np.abs(p.lam0 * p.psi(x) - rhs)) < 1e-12


@pytest.mark.parametrize("c", CS)
def test_unit_norm_and_sign(c):
    p = PSWF(c)
    nrm = integrate.quad(lambda t: float(p.psi(t)) ** 2, -1, 1, epsabs=1e-15, limit=200)[0]
    assert abs(nrm - 1.0) < 1e-12
    assert p.psi0 > 0


@pytest.mark.parametrize("c", CS)
def test_against_scipy_angular(c):
    """Shape agrees with scipy.special.pro_ang1 (an independent implementation)."""
    p = PSWF(c)
    x = np.array([0.0, 0.1, 0.33, 0.5, 0.71, 0.9, 0.98])
    ref = np.array([pro_ang1(0, 0, c, xi)[0] for xi in x])
    assert np.max(np.abs(p.psi(x) / p.psi0 - ref / ref[0])) < 1e-9


@pytest.mark.parametrize("c", [2.0, 9.26, 11.68, 14.08])
def test_eigenvalue_against_scipy_radial(c):
    """lam0 = 2 R_00^(1)(c, 1); R is extrapolated to 1 from just above (SciPy gives NaN at 1)."""
    p = PSWF(c)
    eps = 1e-8
    R, dR = pro_rad1(0, 0, c, 1.0 + eps)
    assert abs(p.lam0 - 2.0 * (R - eps * dR)) < 1e-8


@pytest.mark.parametrize("c", CS)
def test_eigenvalue_at_origin(c):
    """Setting x = 0 in eq. psidefinit gives lam0 psi(0) = 2 C0."""
    p = PSWF(c)
    assert abs(p.lam0 - 2.0 * p.C0 / p.psi0) < 1e-12
    C0q = integrate.quad(lambda t: float(p.psi(t)), 0, 1, epsabs=1e-15)[0]
    assert abs(p.C0 - C0q) < 1e-13


@pytest.mark.parametrize("c", [11.68, 30.0])
def test_extension_is_continuous(c):
    """Beyond |x| = 1 psi is continued by the eigen-equation: value and slope match at 1."""
    p = PSWF(c)
    e = 1e-9
    x = np.array([1.0 - e, 1.0 + e])
    v = p.psi_ext(x)
    d = p.dpsi_ext(x)
    assert abs(v[1] - v[0] - 2 * e * float(p.dpsi(1.0))) < 1e-14
    assert abs(d[0] - d[1]) < 1e-6 * max(1.0, abs(d[0]))


def test_derivative_matches_finite_difference():
    p = PSWF(14.08)
    x = np.linspace(-0.95, 0.95, 11)
    e = 1e-6
    fd = (p.psi(x + e) - p.psi(x - e)) / (2 * e)
    assert np.max(np.abs(fd - p.dpsi(x))) < 1e-8


@pytest.mark.parametrize("delta", [1e-3, 1e-4, 1e-5, 4e-4, 2e-5, 1e-7, 1e-12])
def test_parameter_rule(delta):
    """c solves psi(1)/psi(0) = Delta (Sec. 5.1) and grows roughly like log(1/Delta) (eq. c)."""
    c = c_from_tol(delta)
    p = PSWF(c)
    assert abs(float(p.psi(1.0)) / p.psi0 - delta) < 1e-8 * delta + 1e-15
    assert 0.6 * np.log(1 / delta) < c < 2.0 * np.log(1 / delta)


def test_parameter_rule_monotone():
    cs = [c_from_tol(d) for d in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]
    assert all(a < b for a, b in zip(cs, cs[1:]))
