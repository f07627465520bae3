#!/usr/bin/env python3
"""Error data for the learned parameter proposer, computed with the oracle only.

For seeded synthetic systems of the benchmark kinds (water-shaped,
ionic-liquid-shaped, membrane-shaped; small boxes, since the relative errors
are intensive) and a sweep of ESP parameters (Delta, P, sigma) at rc = 0.9,
this script records the relative errors of the total Coulomb energy, the
diagonal and off-diagonal pressure (the norms of Sec. 5.1) and the RMS force
(reciprocal part from the oracle's gridded ESP, real-space part from the
oracle's direct sums) against classical Ewald.

Output: tests/golden/proposer_data.json (features and log10 errors per row).
Run:    python tests/golden/make_proposer_data.py [--workers 6]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

RC = 0.9
DELTAS = [1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7]
SIGMAS = [0.85, 1.0, 1.15, 1.3]


def systems():
    """(name, kind, builder-args): small boxes of the three workload kinds,
    cubic and triclinic, over a range of densities and sizes."""
    from paper_2601_00161_amd import synth
    out = []
    water_boxes = [(2.6, 100.0), (3.0, 100.0), (2.8, 80.0), (3.2, 120.0), (2.4, 100.0), (3.4, 90.0),
                   (2.5, 110.0), (2.9, 95.0), (3.3, 105.0), (2.7, 85.0), (3.1, 115.0), (3.6, 100.0)]
    for s, (L, dens) in enumerate(water_boxes):
        h = synth.cubic(L)
        if s % 2 == 1:
            rng = np.random.default_rng(500 + s)
            h = h.copy()
            h[0, 1], h[0, 2], h[1, 2] = rng.uniform(-0.2, 0.2, size=3) * L
        nmol = int(round(dens * np.linalg.det(h) / 3))
        out.append((f"water{s}", "water", ("water", nmol, h, 1, 100 + s)))
    for s, L in enumerate([3.6, 4.0, 4.4, 3.4, 3.8, 4.2, 4.6, 3.9]):
        rng = np.random.default_rng(600 + s)
        t = rng.uniform(0.0, 0.15, size=3)
        h = np.array([[L, t[0] * L, t[1] * L], [0.0, L, t[2] * L], [0.0, 0.0, L]])
        npair = int(round(19200 / 16 / 729 * np.linalg.det(h)))
        out.append((f"ionic{s}", "ionic", ("ionic", npair, h, 3, 200 + s)))
    for s, (Lxy, Lz) in enumerate([(3.0, 4.0), (3.4, 4.4), (2.8, 3.8), (3.2, 4.6), (3.6, 4.2), (3.0, 4.8)]):
        out.append((f"membrane{s}", "membrane", ("membrane", Lxy, Lz, 4, 300 + s)))
    return out


def build(spec):
    from paper_2601_00161_amd import synth
    kind = spec[0]
    if kind == "water":
        _, nmol, h, cfg, seed = spec
        return synth.water(nmol, h, config=cfg, seed=seed)
    if kind == "ionic":
        _, npair, h, cfg, seed = spec
        return synth.ionic(npair, h=h, config=cfg, seed=seed)
    _, Lxy, Lz, cfg, seed = spec
    # membrane slab at the config-4 densities: 10 dipole pairs / nm^2 per sheet
    # area and water triplets away from the bilayer
    area = Lxy * Lxy
    nd = int(round(125000 / (25.0 * 25.0) * area))
    nw = int(round(250000 / (25.0 * 25.0 * 14.0) * area * (Lz - 2 * 1.2)))
    h, r, q = synth.membrane(n_dipoles=nd, n_water=nw, L=(Lxy, Lxy, Lz), config=cfg, seed=seed,
                             sheet_offset=0.8, sheet_sigma=0.3, water_gap=1.2)
    return h, r, q


def features(h, q):
    """Features of a system that the error depends on (not N): density of
    charges, mean squared charge, cell anisotropy and tilt."""
    V = abs(np.linalg.det(h))
    n = len(q)
    edges = np.linalg.norm(h, axis=0)
    cosines = [abs(np.dot(h[:, a], h[:, b])) / (edges[a] * edges[b]) for a, b in ((0, 1), (0, 2), (1, 2))]
    return {"log10_density": float(np.log10(n / V)), "log10_q2": float(np.log10(np.mean(q * q))),
            "anisotropy": float(edges.max() / edges.min()), "tilt": float(max(cosines))}


def run_system(item):
    from oracle import esp_direct, esp_grid, ewald
    from oracle.pswf import c_from_tol
    name, kind, spec = item
    h, r, q = build(spec)
    r = r.astype(np.float32).astype(np.float64)
    q = q.astype(np.float32).astype(np.float64)
    ref = ewald.ewald(h, r, q)
    Wr = ref.virial
    diag_ref = np.sqrt(sum(Wr[a, a] ** 2 for a in range(3)))
    off_ref = np.sqrt(sum(Wr[a, b] ** 2 for a, b in ((0, 1), (0, 2), (1, 2))))
    feat = features(h, q)
    rows = []
    for delta in DELTAS:
        c = c_from_tol(delta)
        U_N, W_N, F_N = esp_direct.real_space(h, r, q, c, RC)
        D = int(np.ceil(-np.log10(delta) - 1e-9))
        for P in sorted({max(3, D - 1), max(3, D), D + 1, D + 2}):
            for sigma in SIGMAS:
                M = tuple(max(P, int(np.ceil(sigma * np.linalg.norm(h[:, d]) * c / (np.pi * RC))))
                          for d in range(3))
                g = esp_grid.esp_grid(h, r, q, esp_grid.GridParams(c, c, P, M, RC))
                E = g.energy + U_N
                W = g.virial + W_N
                F = g.forces + F_N
                e_E = abs(E - ref.energy) / abs(ref.energy)
                e_d = np.sqrt(sum((W[a, a] - Wr[a, a]) ** 2 for a in range(3))) / diag_ref
                e_o = np.sqrt(sum((W[a, b] - Wr[a, b]) ** 2 for a, b in ((0, 1), (0, 2), (1, 2)))) / off_ref
                e_F = np.sqrt(np.sum((F - ref.forces) ** 2) / np.sum(ref.forces ** 2))
                rows.append({"system": name, "kind": kind, "n": int(len(q)), **feat,
                             "delta": delta, "P": P, "sigma": sigma, "M": list(M),
                             "log10_err": [float(np.log10(max(v, 1e-16))) for v in (e_E, e_d, e_o, e_F)]})
    print(f"{name}: {len(rows)} rows", flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=6)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "proposer_data.json"))
    args = ap.parse_args()
    items = systems()
    with ProcessPoolExecutor(max_workers=args.workers) as ex:
        rows = [row for rs in ex.map(run_system, items) for row in rs]
    meta = {"rc": RC, "error_order": ["energy", "pressure_diag", "pressure_offdiag", "force_rms"],
            "reference": "classical Ewald (oracle), total Coulomb; ESP reciprocal part = oracle gridded ESP",
            "generator": "tests/golden/make_proposer_data.py"}
    with open(args.out, "w") as f:
        json.dump({"meta": meta, "rows": rows}, f)
    print(f"wrote {len(rows)} rows to {args.out}")


if __name__ == "__main__":
    main()
