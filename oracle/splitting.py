"""PSWF kernel splitting of the Coulomb kernel (paper, Sec. 3.1-3.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

All functions take the splitting bandwidth ``c`` and the cutoff radius ``rc``.
Units: lengths in nm, charges in e, Coulomb constant 1 (energies in e^2/nm).
"""
from __future__ import annotations

import numpy as np

from .pswf import pswf


def phi0(r, c, rc):
    """phi_0^c(r) = (1/C0) int_0^{r/rc} psi(x) dx, equal to 1 for r >= rc (Sec. 3.1)."""
    p = pswf(c)
    r = np.asarray(r, dtype=np.float64)
    x = np.minimum(r / rc, 1.0)
    return p.int_psi(x) / p.C0


def near_kernel(r, c, rc):
    """N^c(r) = (1 - phi0(r))/r for r <= rc, 0 beyond (eq. decomposition)."""
    r = np.asarray(r, dtype=np.float64)
    return np.where(r <= rc, (1.0 - phi0(r, c, rc)) / r, 0.0)


def far_kernel(r, c, rc):
    """F^c(r) = phi0(r)/r (eq. decomposition)."""
    r = np.asarray(r, dtype=np.float64)
    return phi0(r, c, rc) / r


def far_kernel_at_zero(c, rc):
    """lim_{r->0} F^c(r) = psi(0)/(C0 rc) (Sec. 3.1)."""
    p = pswf(c)
    return p.psi0 / (p.C0 * rc)


def near_force_weight(r, c, rc):
    """F_N(r) = 1 - phi0(r) + (r/(C0 rc)) psi(r/rc) for r <= rc, 0 beyond (eq. mathFN).

    The pair force is q_i q_j F_N(r) r_vec / r^3 (eq. Fc).
    """
    p = pswf(c)
    r = np.asarray(r, dtype=np.float64)
    x = np.minimum(r / rc, 1.0)
    val = 1.0 - p.int_psi(x) / p.C0 + (r / (p.C0 * rc)) * p.psi(x)
    return np.where(r <= rc, val, 0.0)


def fourier_prefactor(c):
    """A = 2 pi lambda_0 / C0, the constant in front of the Fourier kernel (eq. UF)."""
    p = pswf(c)
    return 2.0 * np.pi * p.lam0 / p.C0


def far_hat(kabs, c, rc, extend=False):
    """Fourier kernel  F^c_hat(k) = (2 pi lam0/C0) psi(|k| rc/c)/|k|^2  (eq. UF).

    The formula holds for |k| <= c/rc.  With ``extend`` the PSWF is continued
    beyond its band by the eigen-equation, which gives the exact transform of
    F^c for every k; otherwise modes beyond c/rc are returned as zero, the
    truncation stated after eq. Far.
    """
    p = pswf(c)
    k = np.asarray(kabs, dtype=np.float64)
    x = k * rc / c
    A = fourier_prefactor(c)
    if extend:
        safe = np.where(k > 0, k, 1.0)
        return np.where(k > 0, A * p.psi_ext(x) / (safe * safe), 0.0)
    inside = (x <= 1.0) & (k > 0)
    out = np.zeros_like(k)
    out[inside] = A * p.psi(x[inside]) / (k[inside] ** 2)
    return out


def pressure_kernel(kvec, c, rc):
    """Mode-wise pressure kernel P^c_hat(k), a 3x3 tensor per mode (Sec. 4.1).

        P_hat = F_hat (I - 2 k k^T/|k|^2) + A (|k| rc/c) psi'(|k| rc/c)/|k|^4 k k^T

    for 0 < |k| <= c/rc and zero beyond (truncation after eq. Far).  The sign
    of the long-range tensor is the one of eq. UFPree, +1/(2 det(h)^2); the
    printed -1/(2 det h) of eq. Far is read as a slip.

    kvec: (..., 3).  Returns (..., 3, 3).
    """
    p = pswf(c)
    kvec = np.asarray(kvec, dtype=np.float64)
    k2 = np.einsum("...i,...i->...", kvec, kvec)
    k = np.sqrt(k2)
    x = k * rc / c
    inside = (x <= 1.0) & (k > 0)
    A = fourier_prefactor(c)
    F = np.zeros_like(k)
    D = np.zeros_like(k)
    F[inside] = A * p.psi(x[inside]) / k2[inside]
    D[inside] = A * x[inside] * p.dpsi(x[inside]) / (k2[inside] ** 2)
    kk = np.einsum("...i,...j->...ij", kvec, kvec)
    eye = np.eye(3)
    safe_k2 = np.where(inside, k2, 1.0)
    return (F[..., None, None] * (eye - 2.0 * kk / safe_k2[..., None, None])
            + D[..., None, None] * kk)


def self_energy(q, c, rc):
    """U_self = -(psi(0)/(2 C0 rc)) sum q^2 (eq. selfen)."""
    p = pswf(c)
    q = np.asarray(q, dtype=np.float64)
    return -p.psi0 / (2.0 * p.C0 * rc) * float(np.sum(q * q))


def background_integral(c, rc, nquad=200):
    """I_c = rc^2/2 - int_0^rc r phi0(r) dr, by Gauss-Legendre quadrature (Sec. 3.4)."""
    t, w = np.polynomial.legendre.leggauss(nquad)
    r = 0.5 * rc * (t + 1.0)
    return 0.5 * rc * rc - 0.5 * rc * float(np.sum(w * r * phi0(r, c, rc)))


def background_correction(q, V, c, rc):
    """Charge-background and background-background terms for Q != 0 (eq. Corr).

    Returns (U_cb + U_bb, W_corr) where W_corr = V (P_cb + P_bb) is the 3x3
    virial in energy units; both are isotropic.
    """
    Q = float(np.sum(np.asarray(q, dtype=np.float64)))
    Ic = background_integral(c, rc)
    U_cb = -4.0 * np.pi * Q * Q / V * Ic
    U_bb = 2.0 * np.pi * Q * Q / V * Ic
    P_cb = -4.0 * np.pi * Q * Q / V ** 2 * Ic
    P_bb = 2.0 * np.pi * Q * Q / V ** 2 * Ic
    return U_cb + U_bb, V * (P_cb + P_bb) * np.eye(3)
