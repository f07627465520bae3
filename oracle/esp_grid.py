"""Gridded ESP: the particle-mesh method of the paper written out plainly.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Sec. 4.1 (Algorithm 1: spreading, forward FFT, diagonal scaling,
Fourier collection), the PSWF window of Sec. 4.2, the stencil of Sec. 4.3
and the analytic-differentiation force path of App. C (eq. UFAnal, eq. AD).

Readings taken where the paper is silent or inconsistent:

* The grid lies along the cell vectors: M_d subintervals of cell vector d,
  grid coordinates u = M s.  The window is separable in grid coordinates, so
  for a triclinic cell its transform is prod_d w_hat(2 pi m_d / M_d).  Sec. 4.2
  states only the orthorhombic case.
* Stencil: the P grid points g0 + p, p = 0..P-1, with g0 = ceil(u - P/2).
  This is the "P closest grid points" of Sec. 4.3 for odd and even P alike.
* The window is W(x) = psi_0^{c_spread}(x / omega) with omega = P/2 in grid
  units, and its transform w_hat(kappa) = omega lam0 psi(omega kappa / c)
  (Sec. 4.2); beyond the band psi is continued by its eigen-equation, which
  keeps w_hat the exact transform of the compactly supported window.
* Modes: every m != 0 with |k| <= c_split/rc contributes; all other modes
  are dropped (truncation after eq. Far; tin-foil boundary, eq. UF).
* Forces: F_i = -q_i h^{-T} diag(M) sum_g phi[g] grad_u W(u_i - g), where
  phi is the unnormalised inverse FFT of F_hat rho_hat / (V W_hat^2).  The
  factor 1/2 printed in eq. AD is read as a slip: the energy is a quadratic
  form in the grid charges, whose derivative carries a factor 2.
* The reported energy is U_F + U_self (+ the background terms of eq. Corr),
  the "k-space energy" of an MD code; the virial is V * (P_F + P_corr).

The FFT is numpy's full complex transform (sign exp(-2 pi i m.g/M)); no
half-spectrum symmetry is used.

`local_virial` is the per-particle split of the Fourier virial (Sec. 4.4,
eq. rhodiag, eq. PinsFind): Pi = inverse FFT of P_hat rho_hat / W_hat^2 per
tensor component, gathered with the plain window and scaled by q_i / (2V),
so that the shares add up to W_F exactly on the grid (the spreading weights
are a partition of the grid charge).  The background term of eq. Corr is not
split.

`esp_grid_ik` is the other force option of App. C, ik-differentiation
(eq. rhodiagforce): the field i k F_hat rho_hat / (V W_hat^2) is brought back
by three inverse FFTs and gathered with the plain window.  Reading: a mode
whose index is the Nyquist index M_d/2 of an even M_d has no partner -m_d,
so its i k_d term is not the transform of a real field; such modes are
dropped from the field (with the grid rule they lie outside the cutoff
sphere anyway), which keeps the net force exactly zero.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lattice, splitting
from .pswf import pswf


@dataclass
class GridParams:
    c_split: float
    c_spread: float
    P: int
    M: tuple
    rc: float


@dataclass
class GridResult:
    energy: float              # U_F + U_self + U_corr
    virial: np.ndarray         # 3x3, V * (P_F + P_corr)
    forces: np.ndarray | None  # F_F, (N, 3)
    U_F: float
    U_self: float
    U_corr: float
    rho_grid: np.ndarray       # spread charges, shape (M1, M2, M3), index [g1, g2, g3]
    phi_grid: np.ndarray | None


def grid_coordinates(h, r, M):
    """u = M * s with s = h^{-1} r wrapped into [0, 1)."""
    s = lattice.reduced(h, r)
    s = s - np.floor(s)
    return s * np.asarray(M, np.float64)


def stencil(u, P, c_spread):
    """Base index g0 = ceil(u - P/2) and window values/derivatives at g0 + p.

    Returns (g0, w, dw) with g0 of shape (N, 3) (integers, may be negative
    before wrapping) and w, dw of shape (N, 3, P):  w = W(u - g0 - p) and
    dw = dW/du at the same points, W(x) = psi(x / omega), omega = P/2.
    """
    p = pswf(c_spread)
    omega = P / 2.0
    g0 = np.ceil(u - P / 2.0)
    x = u[:, :, None] - g0[:, :, None] - np.arange(P)[None, None, :]
    w = p.psi(x / omega)
    dw = p.dpsi(x / omega) / omega
    return g0.astype(np.int64), w, dw


def window_hat(M, P, c_spread):
    """w_hat(2 pi m / M) for the DFT indices m = 0..M-1 (signed m = m - M if m >= M/2)."""
    p = pswf(c_spread)
    omega = P / 2.0
    m = np.fft.fftfreq(M, d=1.0 / M)                 # signed integers
    kappa = 2.0 * np.pi * m / M
    return omega * p.lam0 * p.psi_ext(omega * kappa / c_spread)


def spread(h, r, q, prm: GridParams):
    """Step 1: rho_grid[g] = sum_j q_j prod_d W(u_jd - g_d), periodised (eq. gridding)."""
    M = np.asarray(prm.M, dtype=np.int64)
    u = grid_coordinates(h, r, M)
    g0, w, _ = stencil(u, prm.P, prm.c_spread)
    q = np.asarray(q, np.float64)
    rho = np.zeros(int(np.prod(M)))
    P = prm.P
    for a in range(P):
        ia = (g0[:, 0] + a) % M[0]
        for b in range(P):
            ib = (g0[:, 1] + b) % M[1]
            wab = q * w[:, 0, a] * w[:, 1, b]
            for cc in range(P):
                ic = (g0[:, 2] + cc) % M[2]
                idx = (ia * M[1] + ib) * M[2] + ic
                rho += np.bincount(idx, weights=wab * w[:, 2, cc], minlength=rho.size)
    return rho.reshape(tuple(M))


def mode_weights(h, prm: GridParams):
    """Per-mode arrays on the full DFT grid: k vectors, mask, W_hat^2, F_hat, P_hat."""
    M = prm.M
    axes = [np.fft.fftfreq(Md, d=1.0 / Md) for Md in M]
    m = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    k = m @ lattice.recip_matrix(h).T
    kabs = np.sqrt(np.einsum("...i,...i->...", k, k))
    wh = [window_hat(Md, prm.P, prm.c_spread) for Md in M]
    What = wh[0][:, None, None] * wh[1][None, :, None] * wh[2][None, None, :]
    Fhat = splitting.far_hat(kabs, prm.c_split, prm.rc)      # 0 at m = 0 and beyond c/rc
    Phat = splitting.pressure_kernel(k, prm.c_split, prm.rc)
    return k, What, Fhat, Phat


def esp_grid(h, r, q, prm: GridParams, forces=True):
    """Energy, virial and forces of the reciprocal-space ESP path."""
    h = np.asarray(h, np.float64)
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    M = np.asarray(prm.M, dtype=np.int64)

    rho = spread(h, r, q, prm)                                # Step 1
    rho_hat = np.fft.fftn(rho)                                # Step 2
    k, What, Fhat, Phat = mode_weights(h, prm)
    e = np.abs(rho_hat) ** 2 / What ** 2                      # Step 3
    U_F = float(np.sum(Fhat * e)) / (2.0 * V)                 # Step 4
    W_F = np.einsum("abc,abcij->ij", e, Phat) / (2.0 * V)

    U_self = splitting.self_energy(q, prm.c_split, prm.rc)
    U_corr, W_corr = splitting.background_correction(q, V, prm.c_split, prm.rc)

    F = None
    phi = None
    if forces:
        G = Fhat / (V * What ** 2)
        phi = np.real(np.fft.ifftn(G * rho_hat)) * float(np.prod(M))
        u = grid_coordinates(h, r, M)
        g0, w, dw = stencil(u, prm.P, prm.c_spread)
        grad = np.zeros((r.shape[0], 3))
        P = prm.P
        for a in range(P):
            ia = (g0[:, 0] + a) % M[0]
            for b in range(P):
                ib = (g0[:, 1] + b) % M[1]
                for cc in range(P):
                    ic = (g0[:, 2] + cc) % M[2]
                    ph = phi[ia, ib, ic]
                    grad[:, 0] += ph * dw[:, 0, a] * w[:, 1, b] * w[:, 2, cc]
                    grad[:, 1] += ph * w[:, 0, a] * dw[:, 1, b] * w[:, 2, cc]
                    grad[:, 2] += ph * w[:, 0, a] * w[:, 1, b] * dw[:, 2, cc]
        hinvT = np.linalg.inv(h).T
        F = -q[:, None] * ((grad * M[None, :].astype(np.float64)) @ hinvT.T)
    return GridResult(U_F + U_self + U_corr, W_F + W_corr, F, U_F, U_self, U_corr, rho, phi)


def nyquist_mask(M):
    """False on modes with m_d = -M_d/2 for an even M_d (full DFT grid)."""
    keep = np.ones(tuple(int(m) for m in M), dtype=bool)
    for d, Md in enumerate(M):
        if Md % 2 == 0:
            sl = [slice(None)] * 3
            sl[d] = Md // 2
            keep[tuple(sl)] = False
    return keep


def esp_grid_ik(h, r, q, prm: GridParams):
    """Energy, virial and ik-differentiated forces (App. C, eq. rhodiagforce):
    F_i = -q_i sum_g W(u_i - g) E(g), E = unnormalised inverse FFT of
    i k F_hat rho_hat / (V W_hat^2)."""
    h = np.asarray(h, np.float64)
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    M = np.asarray(prm.M, dtype=np.int64)
    base = esp_grid(h, r, q, prm, forces=False)
    rho_hat = np.fft.fftn(base.rho_grid)
    k, What, Fhat, _ = mode_weights(h, prm)
    G = Fhat / (V * What ** 2) * nyquist_mask(M)
    u = grid_coordinates(h, r, M)
    g0, w, _ = stencil(u, prm.P, prm.c_spread)
    F = np.zeros((r.shape[0], 3))
    P = prm.P
    for a in range(3):
        E = np.real(np.fft.ifftn(1j * k[..., a] * G * rho_hat)) * float(np.prod(M))
        acc = np.zeros(r.shape[0])
        for i1 in range(P):
            ia = (g0[:, 0] + i1) % M[0]
            for i2 in range(P):
                ib = (g0[:, 1] + i2) % M[1]
                for i3 in range(P):
                    ic = (g0[:, 2] + i3) % M[2]
                    acc += E[ia, ib, ic] * w[:, 0, i1] * w[:, 1, i2] * w[:, 2, i3]
        F[:, a] = -q * acc
    return GridResult(base.energy, base.virial, F, base.U_F, base.U_self, base.U_corr, base.rho_grid, None)


def local_virial(h, r, q, prm: GridParams):
    """Per-particle Fourier virial W^i (N, 3, 3): q_i / (2V) sum_g W(u_i - g) Pi(g),
    Pi = unnormalised inverse FFT of P_hat rho_hat / W_hat^2 (eq. rhodiag, eq. PinsFind)."""
    h = np.asarray(h, np.float64)
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    M = np.asarray(prm.M, dtype=np.int64)
    rho_hat = np.fft.fftn(spread(h, r, q, prm))
    _, What, _, Phat = mode_weights(h, prm)
    u = grid_coordinates(h, r, M)
    g0, w, _ = stencil(u, prm.P, prm.c_spread)
    out = np.zeros((r.shape[0], 3, 3))
    P = prm.P
    for a in range(3):
        for b in range(a, 3):
            Pi = np.real(np.fft.ifftn(Phat[..., a, b] / What ** 2 * rho_hat)) * float(np.prod(M))
            acc = np.zeros(r.shape[0])
            for i1 in range(P):
                ia = (g0[:, 0] + i1) % M[0]
                for i2 in range(P):
                    ib = (g0[:, 1] + i2) % M[1]
                    for i3 in range(P):
                        ic = (g0[:, 2] + i3) % M[2]
                        acc += Pi[ia, ib, ic] * w[:, 0, i1] * w[:, 1, i2] * w[:, 2, i3]
            out[:, a, b] = out[:, b, a] = q * acc / (2.0 * V)
    return out
