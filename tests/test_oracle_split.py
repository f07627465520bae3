"""Pins of the oracle's PSWF kernel split (paper, Sec. 3.1-3.4)."""
import numpy as np
import pytest
from scipy import integrate

from oracle import splitting
from oracle.pswf import PSWF, c_from_tol

RC = 0.9
CS = [c_from_tol(1e-4), c_from_tol(1e-6), 25.0]


@pytest.mark.parametrize("c", CS)
def test_split_is_exact_and_compact(c):
    """N^c + F^c = 1/r for r > 0, and N^c(rc) = 0 (Sec. 3.1)."""
    r = np.linspace(0.01, 2.0, 97)
    total = splitting.near_kernel(r, c, RC) + splitting.far_kernel(r, c, RC)
    assert np.max(np.abs(total * r - 1.0)) < 1e-13
    assert abs(float(splitting.near_kernel(np.array([RC]), c, RC)[0])) < 1e-14
    assert np.all(splitting.near_kernel(np.array([RC * 1.0001, 1.5]), c, RC) == 0.0)


@pytest.mark.parametrize("c", CS)
def test_far_kernel_limit_at_origin(c):
    r = np.array([1e-7])
    assert abs(float(splitting.far_kernel(r, c, RC)[0]) - splitting.far_kernel_at_zero(c, RC)) < 1e-6


@pytest.mark.parametrize("c", CS)
def test_force_weight_is_minus_r2_dN_dr(c):
    """The pair-force weight F_N of eq. mathFN equals -r^2 dN^c/dr inside rc."""
    r = np.linspace(0.05, 0.89, 15)
    e = 1e-6
    dN = (splitting.near_kernel(r + e, c, RC) - splitting.near_kernel(r - e, c, RC)) / (2 * e)
    assert np.max(np.abs(-r * r * dN - splitting.near_force_weight(r, c, RC))) < 1e-7


@pytest.mark.parametrize("c", CS)
def test_fourier_kernel_is_radial_transform(c):
    """F_hat(k) of eq. UF equals the radial transform (App. A.4) of F^c.

    Written as 4 pi/k^2 minus the transform of the compactly supported N^c,
    so that the quadrature is over [0, rc] only.
    """
    p = PSWF(c)
    for k in np.linspace(0.3, 0.999 * c / RC, 9):
        nhat = 4 * np.pi * integrate.quad(
            lambda r: float(splitting.near_kernel(np.array([r]), c, RC)[0]) * np.sin(k * r) / (k * r) * r * r,
            0.0, RC, epsabs=1e-14, epsrel=1e-12, limit=400)[0]
        ref = 4 * np.pi / k ** 2 - nhat
        got = float(splitting.far_hat(np.array([k]), c, RC)[0])
        assert abs(got - ref) < 1e-10 * max(1.0, abs(ref))
    # beyond the band the truncated kernel is zero, the extended one is not
    kb = np.array([1.2 * c / RC])
    assert splitting.far_hat(kb, c, RC)[0] == 0.0
    assert splitting.far_hat(kb, c, RC, extend=True)[0] != 0.0
    # k -> 0: F_hat k^2 / 4 pi -> 1 (the Coulomb limit)
    k0 = np.array([1e-4])
    assert abs(float(splitting.far_hat(k0, c, RC)[0]) * 1e-8 / (4 * np.pi) - 1) < 1e-6
    assert p.C0 > 0


@pytest.mark.parametrize("c", CS)
def test_pressure_kernel_is_strain_derivative(c):
    """P_hat = F_hat I + 2 (dF_hat/d|k|^2) k k^T (eq. UFPree): checked by a finite
    difference of F_hat in |k|^2, independent of the closed form after eq. UFPree."""
    rng = np.random.default_rng(3)
    kv = rng.normal(size=(20, 3))
    kv *= (rng.uniform(0.2, 0.95, size=20) * c / RC / np.linalg.norm(kv, axis=1))[:, None]
    k2 = np.sum(kv * kv, axis=1)
    e = 1e-5 * k2
    Fp = splitting.far_hat(np.sqrt(k2 + e), c, RC)
    Fm = splitting.far_hat(np.sqrt(k2 - e), c, RC)
    dF = (Fp - Fm) / (2 * e)
    F = splitting.far_hat(np.sqrt(k2), c, RC)
    ref = F[:, None, None] * np.eye(3) + 2 * dF[:, None, None] * np.einsum("ni,nj->nij", kv, kv)
    got = splitting.pressure_kernel(kv, c, RC)
    scale = np.max(np.abs(ref), axis=(1, 2))
    assert np.max(np.max(np.abs(got - ref), axis=(1, 2)) / scale) < 5e-6


def test_background_integral_matches_quadrature():
    c = CS[0]
    ref = integrate.quad(lambda r: r * (1 - float(splitting.phi0(np.array([r]), c, RC)[0])), 0, RC,
                         epsabs=1e-15)[0]
    assert abs(splitting.background_integral(c, RC) - ref) < 1e-13


def test_self_energy_value():
    c = CS[0]
    q = np.array([1.0, -0.5, -0.5])
    p = PSWF(c)
    assert abs(splitting.self_energy(q, c, RC) + p.psi0 / (2 * p.C0 * RC) * 1.5) < 1e-14
