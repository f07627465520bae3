"""Cell algebra, explicit structure factors and periodic neighbour pairs.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Conventions (paper, Sec. 2.2 and 3.2): the cell matrix h has the cell vectors
as columns, r = h s with reduced coordinates s, V = det h, and reciprocal
vectors k = 2 pi h^{-T} m for integer m.  The structure factor is
rho(k) = sum_j q_j exp(i k.r_j) = sum_j q_j exp(2 pi i m.s_j).
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import cKDTree


def volume(h):
    return float(np.linalg.det(np.asarray(h, dtype=np.float64)))


def reduced(h, r):
    """s = h^{-1} r for every row of r (not wrapped)."""
    return np.linalg.solve(np.asarray(h, np.float64), np.asarray(r, np.float64).T).T


def recip_matrix(h):
    """B = 2 pi h^{-T}, so that k = B m (eq. vector)."""
    return 2.0 * np.pi * np.linalg.inv(np.asarray(h, np.float64)).T


def perpendicular_widths(h):
    """Distance between opposite faces of the cell, one per cell vector."""
    h = np.asarray(h, np.float64)
    V = abs(np.linalg.det(h))
    a, b, c = h[:, 0], h[:, 1], h[:, 2]
    return np.array([V / np.linalg.norm(np.cross(b, c)),
                     V / np.linalg.norm(np.cross(c, a)),
                     V / np.linalg.norm(np.cross(a, b))])


def mode_box(h, kcut):
    """Half-widths mmax_d so that every |k| <= kcut has |m_d| <= mmax_d.

    m_d = h_d . k / (2 pi), so the bound is kcut |h_d| / (2 pi).
    """
    h = np.asarray(h, np.float64)
    return np.ceil(kcut * np.linalg.norm(h, axis=0) / (2.0 * np.pi)).astype(int)


def mode_vectors(h, mmax):
    """Integer modes m on the box [-mmax, mmax]^3 and k = 2 pi h^{-T} m.

    Returns (m, k) with shapes (n1, n2, n3, 3); axis d runs over m_d from
    -mmax_d to mmax_d.
    """
    axes = [np.arange(-int(M), int(M) + 1) for M in mmax]
    m = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).astype(np.float64)
    k = m @ recip_matrix(h).T
    return m, k


def _phases(s, mmax):
    """exp(2 pi i m s_d) for m in [-mmax_d, mmax_d], one (N, 2 mmax_d + 1) array per d."""
    out = []
    for d in range(3):
        m = np.arange(-int(mmax[d]), int(mmax[d]) + 1)
        out.append(np.exp(2j * np.pi * np.multiply.outer(s[:, d], m)))
    return out


def structure_factor(h, r, q, mmax):
    """rho(k) = sum_j q_j exp(2 pi i m.s_j) on the mode box (Sec. 3.2).

    The three-dimensional phase factorises over the reduced coordinates, so
    the sum is evaluated one m_1 slab at a time as a matrix product.
    """
    s = reduced(h, r)
    q = np.asarray(q, np.float64)
    A1, A2, A3 = _phases(s, mmax)
    S = np.empty((A1.shape[1], A2.shape[1], A3.shape[1]), dtype=np.complex128)
    for a in range(A1.shape[1]):
        S[a] = ((q * A1[:, a])[:, None] * A2).T @ A3
    return S


def back_transform(h, r, X, mmax):
    """T_i = sum_m X(m) exp(-2 pi i m.s_i) for every particle i.

    X has shape (ncomp, n1, n2, n3); returns (N, ncomp) complex.  Used for the
    per-particle Fourier sums of the force expression (eq. Fc).
    """
    s = reduced(h, r)
    A1, A2, A3 = (np.conj(a) for a in _phases(s, mmax))
    ncomp = X.shape[0]
    T = np.zeros((s.shape[0], ncomp), dtype=np.complex128)
    for a in range(A1.shape[1]):
        # Y[i, c, b] = sum_m3 conj(A3[i, m3]) X[c, a, b, m3]
        Xa = X[:, a]
        Y = (A3 @ Xa.reshape(-1, Xa.shape[-1]).T).reshape(s.shape[0], ncomp, Xa.shape[1])
        T += A1[:, a][:, None] * np.einsum("ib,icb->ic", A2, Y)
    return T


def pair_chunks(h, r, rcut, chunk=2048, rows=None):
    """Periodic pairs (i, j, n) with 0 < |r_i - r_j - h n| <= rcut, in chunks of i.

    Positions are wrapped into the cell, the images that can reach the cell
    are replicated explicitly, and SciPy's k-d tree returns the pairs.  Every
    ordered pair appears once per image, so sums over the result carry the
    factor 1/2 of the primed double sums of the paper.  ``rows`` restricts i
    to a subset of particles.

    Yields (i, j, d) with d = r_i - (r_j + h n) of shape (npairs, 3).
    """
    h = np.asarray(h, np.float64)
    s = reduced(h, r)
    s = s - np.floor(s)
    r0 = s @ h.T
    N = r0.shape[0]
    nimg = np.ceil(rcut / perpendicular_widths(h)).astype(int)
    shifts = np.array(list(itertools.product(*[range(-n, n + 1) for n in nimg])), dtype=np.float64)
    ext = (r0[None, :, :] + (shifts @ h.T)[:, None, :]).reshape(-1, 3)
    tree = cKDTree(ext)
    idx = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    for c0 in range(0, idx.size, chunk):
        sel = idx[c0:c0 + chunk]
        sub = cKDTree(r0[sel])
        res = sub.sparse_distance_matrix(tree, rcut, output_type="ndarray")
        keep = res["v"] > 0.0
        ii = sel[res["i"][keep].astype(np.int64)]
        jj = res["j"][keep].astype(np.int64)
        yield ii, jj % N, r0[ii] - ext[jj]


def pairs_within(h, r, rcut, chunk=2048):
    """All pairs of ``pair_chunks`` concatenated (small systems only)."""
    I, J, D = zip(*pair_chunks(h, r, rcut, chunk))
    return np.concatenate(I), np.concatenate(J), np.concatenate(D)
