"""ESP with explicit structure-factor sums (paper, Sec. 3, App. C).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Evaluates the three pieces of eq. splitting directly:

* U_N  -- eq. UN, real-space pairs within rc with the kernel N^c;
* U_F  -- eq. UF, the Fourier sum over 0 < |k| <= c/rc (the truncation
          stated after eq. Far) with rho(k) summed explicitly;
* U_self -- eq. selfen;

plus the background terms of eq. Corr when the net charge is non-zero.
Virials (V * P) follow eq. PinsN for the real-space part, with the sign
+1/2 that eq. pressuretensor implies (the printed -1/2 is read as a slip), and
eq. UFPree / Sec. 4.1 (P^c_hat) for the Fourier part.  Forces follow eq. Fc.

No spreading, grid or FFT is involved: this isolates the error of the split
itself from the error of the particle-mesh discretisation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lattice, splitting


@dataclass
class SplitResult:
    """Energies and virials of the split, kept separate so tests can combine them."""
    U_N: float
    U_F: float
    U_self: float
    U_corr: float
    W_N: np.ndarray
    W_F: np.ndarray
    W_corr: np.ndarray
    F_N: np.ndarray | None
    F_F: np.ndarray | None

    @property
    def energy(self):
        return self.U_N + self.U_F + self.U_self + self.U_corr

    @property
    def virial(self):
        return self.W_N + self.W_F + self.W_corr

    @property
    def forces(self):
        return None if self.F_N is None else self.F_N + self.F_F


def real_space(h, r, q, c, rc, forces=True):
    """U_N (eq. UN), W_N (eq. PinsN, sign +) and F_N (eq. Fc) over pairs within rc."""
    q = np.asarray(q, np.float64)
    N = q.shape[0]
    U = 0.0
    W = np.zeros((3, 3))
    F = np.zeros((N, 3)) if forces else None
    for i, j, d in lattice.pair_chunks(h, r, rc):
        dist = np.linalg.norm(d, axis=1)
        qq = q[i] * q[j]
        U += 0.5 * float(np.sum(qq * splitting.near_kernel(dist, c, rc)))
        fw = qq * splitting.near_force_weight(dist, c, rc) / dist ** 3
        W += 0.5 * np.einsum("p,pa,pb->ab", fw, d, d)
        if forces:
            for a in range(3):
                F[:, a] += np.bincount(i, weights=fw * d[:, a], minlength=N)
    return U, W, F


def fourier_space(h, r, q, c, rc, forces=True):
    """U_F (eq. UF), W_F (eq. UFPree) and F_F (eq. Fc), truncated at |k| <= c/rc."""
    h = np.asarray(h, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    K = c / rc
    mmax = lattice.mode_box(h, K)
    _, k = lattice.mode_vectors(h, mmax)
    kabs = np.sqrt(np.einsum("...i,...i->...", k, k))
    Fhat = splitting.far_hat(kabs, c, rc)            # zero at k = 0 and beyond c/rc
    Phat = splitting.pressure_kernel(k, c, rc)
    S = lattice.structure_factor(h, r, q, mmax)
    S2 = np.abs(S) ** 2
    U = float(np.sum(Fhat * S2)) / (2.0 * V)
    W = np.einsum("abc,abcij->ij", S2, Phat) / (2.0 * V)
    F = None
    if forces:
        X = np.moveaxis(Fhat[..., None] * k * S[..., None], -1, 0)
        T = lattice.back_transform(h, r, X, mmax)
        F = -(q[:, None] / V) * T.imag
    return U, W, F


def fourier_local_virial(h, r, q, c, rc):
    """Per-particle share of the Fourier-space virial (Sec. 4.4, eq. PinsFind
    with explicit sums): W^i = q_i / (2V) sum_k P_hat(k) Re[exp(-i k.r_i) rho(k)],
    (N, 3, 3).  The shares add up to W_F of `fourier_space`."""
    h = np.asarray(h, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    mmax = lattice.mode_box(h, c / rc)
    _, k = lattice.mode_vectors(h, mmax)
    Phat = splitting.pressure_kernel(k, c, rc)
    S = lattice.structure_factor(h, r, q, mmax)
    X = np.moveaxis((Phat * S[..., None, None]).reshape(S.shape + (9,)), -1, 0)
    T = lattice.back_transform(h, r, X, mmax)
    return (q[:, None] / (2.0 * V) * T.real).reshape(-1, 3, 3)


def esp_direct(h, r, q, c, rc, forces=True):
    """All terms of the PSWF split with explicit Fourier sums."""
    h = np.asarray(h, np.float64)
    r = np.asarray(r, np.float64)
    q = np.asarray(q, np.float64)
    V = lattice.volume(h)
    U_N, W_N, F_N = real_space(h, r, q, c, rc, forces)
    U_F, W_F, F_F = fourier_space(h, r, q, c, rc, forces)
    U_self = splitting.self_energy(q, c, rc)
    U_corr, W_corr = splitting.background_correction(q, V, c, rc)
    return SplitResult(U_N, U_F, U_self, U_corr, W_N, W_F, W_corr, F_N, F_F)
