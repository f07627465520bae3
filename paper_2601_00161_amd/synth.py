"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates positions, charges and cells only; it holds none of the
ESP arithmetic and is shared by the tests, the benchmark and the CPU oracle
checks.  Every generator is deterministic in (config, seed):
``numpy.random.Generator(PCG64(20260101 + 100 * config + seed))``.

Units: nm and e.  Cells are 3x3 matrices whose columns are the cell vectors
(h[i, j] = component i of vector j).  Every system is neutral in FP64 by
construction.

Stand-ins (the paper's equilibrated snapshots and force fields are not
available, so only their shapes are reproduced):

* ``water``     -- rigid 3-site triplets (O -0.8476, H +0.4238 x 2, O-H 0.1 nm,
                   H-O-H 109.47 deg), uniform centres, uniform random
                   orientations: bulk SPC/E-water-shaped (Sec. 5.1-5.2).
* ``ionic``     -- a triclinic cell holding +1 cations and 15-site anions
                   built as seeded self-avoiding walks, partial charges summing
                   to -1: LiTFSI-shaped (Sec. 5.3).
* ``membrane``  -- an orthorhombic slab: two Gaussian sheets of +-0.5 dipole
                   pairs and water triplets elsewhere: bc1-membrane-shaped
                   (Sec. 5.4).
* ``replicas``  -- a batch of small triclinic water-shaped systems.
* ``nacl``      -- rock-salt crystals (cubic 8-ion cell, or the 2-ion FCC
                   primitive cell), for the Madelung check.
"""
from __future__ import annotations

import numpy as np

Q_O, Q_H = -0.8476, 0.4238
R_OH = 0.1
THETA_HOH = np.deg2rad(109.47)


def rng_for(config: int, seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(20260101 + 100 * int(config) + int(seed)))


def cubic(L: float) -> np.ndarray:
    return np.diag([float(L)] * 3)


def random_rotations(rng, n):
    """Uniform random rotation matrices (Shoemake's quaternion method)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1 - u1)
    b = np.sqrt(u1)
    x = a * np.sin(2 * np.pi * u2)
    y = a * np.cos(2 * np.pi * u2)
    z = b * np.sin(2 * np.pi * u3)
    w = b * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _triplet_template():
    half = THETA_HOH / 2
    return np.array([[0.0, 0.0, 0.0],
                     [R_OH * np.sin(half), 0.0, R_OH * np.cos(half)],
                     [-R_OH * np.sin(half), 0.0, R_OH * np.cos(half)]])


def place_triplets(rng, centres):
    """Water-shaped triplets with the given O positions and random orientations."""
    n = centres.shape[0]
    R = random_rotations(rng, n)
    body = np.einsum("nij,aj->nai", R, _triplet_template())
    pos = (centres[:, None, :] + body).reshape(-1, 3)
    q = np.tile([Q_O, Q_H, Q_H], n)
    return pos, q


def water(n_molecules: int, h, config: int = 1, seed: int = 0):
    """n_molecules triplets with uniform fractional centres in cell h."""
    h = np.asarray(h, np.float64)
    rng = rng_for(config, seed)
    s = rng.random((n_molecules, 3))
    centres = s @ h.T
    pos, q = place_triplets(rng, centres)
    return h, pos, q


def config1(seed=0):
    """1,000 triplets in a cubic 3.0 nm cell, N = 3,000."""
    return water(1000, cubic(3.0), config=1, seed=seed)


def config2(seed=0):
    """10,000 triplets in a cubic 6.7 nm cell, N = 30,000."""
    return water(10000, cubic(6.7), config=2, seed=seed)


def ionic_cell():
    """Upper-triangular cell: a = (9,0,0), b = (1.2,9,0), c = (0.8,0.5,9) nm."""
    return np.array([[9.0, 1.2, 0.8],
                     [0.0, 9.0, 0.5],
                     [0.0, 0.0, 9.0]])


def _anion_walk(rng, nsite=15, bond=0.15, min_sep=0.22, tries=200):
    """A self-avoiding 15-site walk with 0.15 nm bonds, sites >= 0.22 nm apart
    unless bonded."""
    for _ in range(tries):
        pts = [np.zeros(3)]
        ok = True
        for _i in range(1, nsite):
            for _t in range(100):
                v = rng.normal(size=3)
                v *= bond / np.linalg.norm(v)
                cand = pts[-1] + v
                d = np.linalg.norm(np.asarray(pts[:-1]) - cand, axis=1) if len(pts) > 1 else np.array([1.0])
                if np.all(d >= min_sep):
                    pts.append(cand)
                    break
            else:
                ok = False
                break
        if ok:
            return np.asarray(pts)
    raise RuntimeError("could not grow a self-avoiding anion")


def ionic(n_pairs: int = 1200, h=None, config: int = 3, seed: int = 0):
    """Cations (+1) and 15-site anions (charges U[-0.7, 1.1] shifted to sum -1)."""
    h = ionic_cell() if h is None else np.asarray(h, np.float64)
    rng = rng_for(config, seed)
    template = _anion_walk(rng)
    template -= template.mean(axis=0)
    qa = rng.uniform(-0.7, 1.1, size=15)
    qa += (-1.0 - qa.sum()) / 15.0
    cat = rng.random((n_pairs, 3)) @ h.T
    centres = rng.random((n_pairs, 3)) @ h.T
    R = random_rotations(rng, n_pairs)
    an = (centres[:, None, :] + np.einsum("nij,aj->nai", R, template)).reshape(-1, 3)
    pos = np.concatenate([cat, an])
    q = np.concatenate([np.ones(n_pairs), np.tile(qa, n_pairs)])
    return h, pos, q


def config3(seed=0):
    return ionic(1200, config=3, seed=seed)


def membrane(n_dipoles: int = 125_000, n_water: int = 250_000, L=(25.0, 25.0, 20.0),
             config: int = 4, seed: int = 0, sheet_offset: float = 2.0, sheet_sigma: float = 0.5,
             water_gap: float = 3.0):
    """Two Gaussian sheets of +-0.5 dipole pairs (centres at the mid-plane +-
    sheet_offset) and water triplets whose centres are at least water_gap
    from the mid-plane."""
    rng = rng_for(config, seed)
    Lx, Ly, Lz = L
    if not water_gap < Lz / 2.0:
        raise ValueError("water_gap must be below half the slab height")
    h = np.diag([Lx, Ly, Lz])
    zc = Lz / 2.0
    half = n_dipoles // 2
    sheets = []
    for sign, n in ((+1, half), (-1, n_dipoles - half)):
        xy = rng.random((n, 2)) * [Lx, Ly]
        z = rng.normal(zc + sign * sheet_offset, sheet_sigma, size=n)
        head = np.column_stack([xy, z + sign * 0.05])     # outward-pointing dipole
        tail = np.column_stack([xy, z - sign * 0.05])
        sheets.append((head, tail))
    pos_d = np.concatenate([np.concatenate([hd, tl]) for hd, tl in sheets])
    q_d = np.concatenate([np.concatenate([np.full(len(hd), 0.5), np.full(len(tl), -0.5)])
                          for hd, tl in sheets])
    centres = np.empty((0, 3))
    while centres.shape[0] < n_water:
        cand = rng.random((2 * n_water + 16, 3)) * [Lx, Ly, Lz]
        cand = cand[np.abs(cand[:, 2] - zc) >= water_gap]
        centres = np.concatenate([centres, cand])
    centres = centres[:n_water]
    pos_w, q_w = place_triplets(rng, centres)
    return h, np.concatenate([pos_d, pos_w]), np.concatenate([q_d, q_w])


def config4(seed=0):
    return membrane(config=4, seed=seed)


def replicas(n_rep: int = 64, config: int = 5, seed: int = 0, n_range=(2000, 60000),
             tols=(1e-3, 1e-4, 1e-5, 1e-6)):
    """Replica batch: per replica (h, pos, q, tol)."""
    rng = rng_for(config, seed)
    out = []
    for _ in range(n_rep):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        n -= n % 3
        V = n / 100.0                                   # water site density, 100 nm^-3
        aspect = rng.uniform(0.8, 1.25, size=3)
        l = aspect * (V / np.prod(aspect)) ** (1.0 / 3.0)
        l = np.clip(l, 3.0, 9.0)
        h = np.diag(l)
        h[0, 1] = rng.uniform(-0.3, 0.3) * l[0]
        h[0, 2] = rng.uniform(-0.3, 0.3) * l[0]
        h[1, 2] = rng.uniform(-0.3, 0.3) * l[1]
        s = rng.random((n // 3, 3))
        pos, q = place_triplets(rng, s @ h.T)
        tol = float(tols[int(rng.integers(0, len(tols)))])
        out.append((h, pos, q, tol))
    return out


def random_neutral(n: int, h, config: int = 0, seed: int = 0):
    """n charges (n even) at uniform positions, charges +-1 scaled, exactly neutral."""
    h = np.asarray(h, np.float64)
    rng = rng_for(config, seed)
    pos = rng.random((n, 3)) @ h.T
    q = rng.uniform(0.2, 1.0, size=n)
    q[1::2] *= -1.0
    q -= q.mean()
    return h, pos, q


def nacl_cubic(a: float = 0.5):
    """Conventional rock-salt cell with edge 2a (a = nearest-neighbour distance), 8 ions."""
    base = np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=np.float64)
    na = base * a
    cl = (base + [1, 0, 0]) * a
    pos = np.concatenate([na, cl]) % (2 * a)
    q = np.concatenate([np.ones(4), -np.ones(4)])
    return np.diag([2 * a] * 3), pos, q


def nacl_primitive(a: float = 0.5):
    """FCC primitive cell (columns (0,a,a), (a,0,a), (a,a,0)): Na at 0, Cl at (a,0,0)."""
    h = np.array([[0.0, a, a],
                  [a, 0.0, a],
                  [a, a, 0.0]])
    pos = np.array([[0.0, 0.0, 0.0], [a, 0.0, 0.0]])
    return h, pos, np.array([1.0, -1.0])
