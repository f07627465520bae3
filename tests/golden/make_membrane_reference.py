#!/usr/bin/env python3
"""Exact total Coulomb energy, virial and sampled forces of the 10^6-charge
membrane-shaped slab, computed with the oracle only.

The system is the seeded synthetic slab (25 x 25 x 20 nm, two Gaussian
sheets of +-0.5 dipole pairs, water-shaped triplets elsewhere; seed 0),
rounded to FP32 as the GPU receives it and converted exactly to FP64.

Direct Ewald sums are out of reach at this size, so the reference is the
oracle's gridded ESP converged to Delta = 1e-12 (P = 13, c from
psi(1)/psi(0) = Delta, grid by the sigma = 1.07 rule on 2,3,5-smooth sizes),
plus the oracle's real-space pair sum at the same c -- the same choice the
paper makes when it measures against a tightly converged mesh method
(Sec. 5.1).  The oracle's CPU tests pin that construction to classical
Ewald on smaller systems: the gridded ESP with a tight window against the
explicit-sum ESP at the same split, and the explicit-sum ESP at
Delta = 1e-13 against converged Ewald.

Output: tests/golden/membrane_1m_reference.json with
  energy, virial (3x3), the relative RMS of the reference forces, and the
  reference forces of SAMPLE particles (indices drawn with a seeded
  generator), so that a GPU result can be scored on all six virial
  components and on a force sample without storing 10^6 force rows.
Run:    python tests/golden/make_membrane_reference.py   (about 15 minutes,
        ~10 GB of memory)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

OUT = os.path.join(ROOT, "tests", "golden", "membrane_1m_reference.json")
DELTA_REF = 1e-12
P_REF = 13
RC = 0.9
SIGMA = 1.07
SAMPLE = 4096
SAMPLE_SEED = 20260104


def smooth(m):
    k = m
    for p in (2, 3, 5):
        while k % p == 0:
            k //= p
    return k == 1


def main():
    from oracle import esp_direct, esp_grid
    from oracle.pswf import c_from_tol
    from paper_2601_00161_amd import synth

    t0 = time.time()
    h, r, q = synth.config4(seed=0)
    r64 = r.astype(np.float32).astype(np.float64)
    q64 = q.astype(np.float32).astype(np.float64)
    N = len(q64)
    c_ref = c_from_tol(DELTA_REF)
    M = []
    for d in range(3):
        m = int(np.ceil(SIGMA * np.linalg.norm(h[:, d]) * c_ref / (np.pi * RC)))
        while not smooth(m):
            m += 1
        M.append(m)
    print(f"N={N} c_ref={c_ref:.6f} P={P_REF} M={M}", flush=True)
    rec = esp_grid.esp_grid(h, r64, q64, esp_grid.GridParams(c_ref, c_ref, P_REF, tuple(M), RC))
    print(f"reciprocal part done ({time.time() - t0:.0f} s)", flush=True)
    U_N, W_N, F_N = esp_direct.real_space(h, r64, q64, c_ref, RC)
    print(f"real-space part done ({time.time() - t0:.0f} s)", flush=True)
    E = rec.energy + U_N
    W = rec.virial + W_N
    F = rec.forces + F_N
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(N, size=SAMPLE, replace=False))
    out = {
        "system": "synth.config4(seed=0): membrane-shaped slab 25x25x20 nm, N=1,000,000, FP32-rounded inputs",
        "reference": f"oracle esp_grid at Delta={DELTA_REF:g} (P={P_REF}, M={M}) + oracle real_space, rc={RC}",
        "delta": DELTA_REF, "c": c_ref, "P": P_REF, "M": M, "rc": RC, "n": int(N),
        "energy": float(E),
        "virial": [[float(x) for x in row] for row in W],
        "energy_parts": {"U_F_self_corr": float(rec.energy), "U_N": float(U_N)},
        "force_rms": float(np.sqrt(np.mean(np.sum(F ** 2, axis=1)))),
        "sample_seed": SAMPLE_SEED,
        "sample_index": [int(i) for i in idx],
        "sample_forces": [[float(x) for x in F[i]] for i in idx],
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
