"""Pins of the classical Ewald reference (paper, Sec. 2.1 and 3.3)."""
import os

import numpy as np
import pytest

from oracle import ewald
from paper_2601_00161_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "nacl_madelung.txt")


def madelung():
    with open(GOLDEN) as f:
        return float([ln for ln in f if not ln.startswith("#") and ln.strip()][0])


TRICLINIC = np.array([[2.0, 0.3, 0.1], [0.0, 2.2, 0.2], [0.0, 0.0, 1.9]])


@pytest.mark.parametrize("cell", [synth.nacl_cubic, synth.nacl_primitive])
def test_nacl_madelung(cell):
    """Both the 8-ion cubic and the 2-ion FCC-primitive (triclinic) cells give
    U = -M * pairs / a, W = U/3 I and zero forces."""
    a = 0.5
    h, r, q = cell(a)
    res = ewald.ewald(h, r, q)
    pairs = len(q) // 2
    assert abs(res.energy / (-pairs / a) - madelung()) < 1e-11
    assert np.max(np.abs(res.virial - res.energy / 3 * np.eye(3))) < 1e-11
    assert np.max(np.abs(res.forces)) < 1e-11


def _system(n=40, seed=1, h=TRICLINIC):
    return synth.random_neutral(n, h, seed=seed)


def test_virial_identity():
    """Coulomb energy is homogeneous of degree -1, so tr W = U (eq. deth)."""
    h, r, q = _system()
    res = ewald.ewald(h, r, q)
    assert abs(np.trace(res.virial) - res.energy) < 1e-10 * abs(res.energy)


def test_net_force_zero():
    h, r, q = _system()
    res = ewald.ewald(h, r, q)
    assert np.max(np.abs(res.forces.sum(axis=0))) < 1e-11


def test_splitting_parameter_independence():
    h, r, q = _system()
    a = ewald.ewald(h, r, q, rcut=0.9)
    b = ewald.ewald(h, r, q, rcut=1.6)
    assert abs(a.energy - b.energy) < 1e-12 * abs(a.energy)
    assert np.max(np.abs(a.virial - b.virial)) < 1e-10
    assert np.max(np.abs(a.forces - b.forces)) < 1e-10


def test_non_neutral_background_is_parameter_independent():
    h, r, q = _system()
    q = q.copy()
    q[0] += 0.37
    a = ewald.ewald(h, r, q, rcut=0.9)
    b = ewald.ewald(h, r, q, rcut=1.6)
    assert abs(a.energy - b.energy) < 1e-11 * abs(a.energy)
    assert np.max(np.abs(a.virial - b.virial)) < 1e-10


def test_forces_are_energy_gradient():
    h, r, q = _system(n=24, seed=2)
    res = ewald.ewald(h, r, q)
    e = 1e-5
    for i in (0, 7, 13):
        for d in range(3):
            rp = r.copy(); rp[i, d] += e
            rm = r.copy(); rm[i, d] -= e
            fd = -(ewald.ewald(h, rp, q, forces=False).energy - ewald.ewald(h, rm, q, forces=False).energy) / (2 * e)
            assert abs(fd - res.forces[i, d]) < 1e-7 * max(1.0, abs(res.forces[i, d]))


def test_virial_is_strain_derivative():
    """W = -dU/d(eps) under r -> (I+eps) r, h -> (I+eps) h at fixed s (eq. instheta)."""
    h, r, q = _system(n=24, seed=3)
    res = ewald.ewald(h, r, q)
    e = 1e-6
    W = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3)); eps[a, b] = e
            up = ewald.ewald((np.eye(3) + eps) @ h, r @ (np.eye(3) + eps).T, q, forces=False).energy
            dn = ewald.ewald((np.eye(3) - eps) @ h, r @ (np.eye(3) - eps).T, q, forces=False).energy
            W[a, b] = -(up - dn) / (2 * e)
    assert np.max(np.abs(W - res.virial)) < 1e-7 * np.max(np.abs(res.virial))
