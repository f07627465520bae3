"""Pins of the oracle's ESP (direct sums and gridded), paper Sec. 3-4 and App. C."""
import numpy as np
import pytest

from oracle import esp_direct, esp_grid, ewald, lattice
from oracle.pswf import c_from_tol
from paper_2601_00161_amd import synth

RC = 0.9
TRICLINIC = np.array([[2.0, 0.3, 0.1], [0.0, 2.2, 0.2], [0.0, 0.0, 1.9]])


def rel_rms(a, b):
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


@pytest.fixture(scope="module")
def sysA():
    h, r, q = synth.random_neutral(60, TRICLINIC, seed=1)
    return h, r, q, ewald.ewald(h, r, q)


def test_direct_esp_converges_to_ewald(sysA):
    """With Delta -> 1e-13 the split is exact: U, W, F equal converged Ewald."""
    h, r, q, ref = sysA
    res = esp_direct.esp_direct(h, r, q, c_from_tol(1e-13), RC)
    assert abs(res.energy - ref.energy) < 1e-12 * abs(ref.energy)
    assert np.max(np.abs(res.virial - ref.virial)) < 1e-11 * np.max(np.abs(ref.virial))
    assert rel_rms(res.forces, ref.forces) < 1e-12


@pytest.mark.parametrize("delta", [1e-4, 1e-6])
def test_direct_esp_error_is_order_delta(sysA, delta):
    h, r, q, ref = sysA
    res = esp_direct.esp_direct(h, r, q, c_from_tol(delta), RC)
    assert abs(res.energy - ref.energy) / abs(ref.energy) < 10 * delta
    assert np.max(np.abs(res.virial - ref.virial)) / np.max(np.abs(ref.virial)) < 10 * delta
    assert rel_rms(res.forces, ref.forces) < 10 * delta
    # the truncation at c/rc breaks the virial identity only at O(Delta),
    # measured against the largest term of the split
    scale = max(abs(res.U_F), abs(res.U_self), abs(res.U_N))
    assert abs(np.trace(res.virial) - res.energy) / scale < 10 * delta


def test_non_neutral_correction_matches_ewald_background(sysA):
    """eq. Corr reproduces the neutralising-background energy and virial of Ewald."""
    h, r, q, _ = sysA
    q = q.copy()
    q[0] += 0.3
    ref = ewald.ewald(h, r, q)
    res = esp_direct.esp_direct(h, r, q, c_from_tol(1e-13), RC)
    assert res.U_corr != 0.0
    assert abs(res.energy - ref.energy) < 1e-12 * abs(ref.energy)
    assert np.max(np.abs(res.virial - ref.virial)) < 1e-10 * np.max(np.abs(ref.virial))


def _grid_params(h, c_split, c_spread, P, sigma):
    M = tuple(int(np.ceil(sigma * np.linalg.norm(h[:, d]) * c_split / (np.pi * RC))) for d in range(3))
    return esp_grid.GridParams(c_split, c_spread, P, M, RC)


def test_gridded_converges_to_direct(sysA):
    """Refining the window (c_spread, P) and the grid drives the gridded Fourier
    part to the direct-sum Fourier part: the spreading, FFT, deconvolution,
    triclinic mode vectors and force gather are all pinned by this."""
    h, r, q, _ = sysA
    c = c_from_tol(1e-6)
    U_F, W_F, F_F = esp_direct.fourier_space(h, r, q, c, RC)
    prm = _grid_params(h, c, c_from_tol(1e-13), 16, 2.0)
    g = esp_grid.esp_grid(h, r, q, prm)
    assert abs(g.U_F - U_F) < 1e-12 * abs(U_F)
    assert np.max(np.abs(g.virial - W_F)) < 1e-12 * np.max(np.abs(W_F))
    assert rel_rms(g.forces, F_F) < 1e-10


@pytest.fixture(scope="module")
def water_small():
    h, r, q = synth.water(40, synth.cubic(1.9), config=1, seed=7)
    h = h.copy()
    h[0, 1] = 0.25
    h[1, 2] = -0.15
    c = c_from_tol(1e-4)
    return h, r, q, _grid_params(h, c, c, 5, 1.07)


def test_gridded_forces_are_exact_gradient(water_small):
    """Analytic differentiation gives the exact gradient of the gridded energy
    (App. C), which pins the factor of eq. AD."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid(h, r, q, prm)
    e = 1e-6
    for i in (0, 11, 50, 101):
        for d in range(3):
            rp = r.copy(); rp[i, d] += e
            rm = r.copy(); rm[i, d] -= e
            fd = -(esp_grid.esp_grid(h, rp, q, prm, forces=False).energy
                   - esp_grid.esp_grid(h, rm, q, prm, forces=False).energy) / (2 * e)
            assert abs(fd - g.forces[i, d]) < 2e-6 * np.max(np.abs(g.forces))


def test_gridded_virial_is_strain_derivative(water_small):
    """rho_grid depends on s only, so the grid energy's strain derivative is exact."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid(h, r, q, prm, forces=False)
    e = 1e-6
    W = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3)); eps[a, b] = e
            up = esp_grid.esp_grid((np.eye(3) + eps) @ h, r @ (np.eye(3) + eps).T, q, prm, forces=False).energy
            dn = esp_grid.esp_grid((np.eye(3) - eps) @ h, r @ (np.eye(3) - eps).T, q, prm, forces=False).energy
            W[a, b] = -(up - dn) / (2 * e)
    assert np.max(np.abs(W - g.virial)) < 1e-7 * np.max(np.abs(g.virial))


def test_gridded_non_neutral_strain_derivative(water_small):
    h, r, q, prm = water_small
    q = q.copy()
    q[3] += 0.2
    g = esp_grid.esp_grid(h, r, q, prm, forces=False)
    assert g.U_corr != 0
    e = 1e-6
    up = esp_grid.esp_grid((1 + e) * h, r * (1 + e), q, prm, forces=False).energy
    dn = esp_grid.esp_grid((1 - e) * h, r * (1 - e), q, prm, forces=False).energy
    assert abs(-(up - dn) / (2 * e) - np.trace(g.virial)) < 1e-7 * abs(np.trace(g.virial))


def test_parseval(water_small):
    """U_F = 1/2 sum_g phi[g] rho_grid[g] (App. A.3 applied to eq. UFAnal)."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid(h, r, q, prm)
    assert abs(0.5 * np.sum(g.phi_grid * g.rho_grid) - g.U_F) < 1e-12 * abs(g.U_F)


def test_rotation_invariance(water_small):
    """(h, r) -> (R h, R r) leaves s and |k| unchanged: U equal, W -> R W R^T, F -> R F."""
    h, r, q, prm = water_small
    R = synth.random_rotations(np.random.default_rng(5), 1)[0]
    a = esp_grid.esp_grid(h, r, q, prm)
    b = esp_grid.esp_grid(R @ h, r @ R.T, q, prm)
    assert abs(a.energy - b.energy) < 1e-12 * abs(a.energy)
    assert np.max(np.abs(R @ a.virial @ R.T - b.virial)) < 1e-11 * np.max(np.abs(a.virial))
    assert np.max(np.abs(a.forces @ R.T - b.forces)) < 1e-11 * np.max(np.abs(a.forces))


def test_net_force_small_not_zero(water_small):
    """Analytic differentiation does not conserve momentum (App. C): |sum F| is
    small (O(Delta)) but not roundoff."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid(h, r, q, prm)
    n = len(q)
    frms = np.sqrt(np.mean(np.sum(g.forces ** 2, axis=1)))
    ratio = np.linalg.norm(g.forces.sum(axis=0)) / (np.sqrt(n) * frms)
    assert ratio < 1e-3


def test_paper_parameter_set_accuracy():
    """At the paper's standard setting (Delta = 4e-4, P = 5, spacing ~0.26 nm,
    rc = 0.9) the total Coulomb force error lands near 4e-4 (Sec. 5.2)."""
    h, r, q = synth.water(300, synth.cubic(2.1), config=1, seed=3)
    ref = ewald.ewald(h, r, q)
    c = c_from_tol(4e-4)
    M = tuple([int(round(2.1 / 0.26))] * 3)
    prm = esp_grid.GridParams(c, c, 5, M, RC)
    g = esp_grid.esp_grid(h, r, q, prm)
    U_N, W_N, F_N = esp_direct.real_space(h, r, q, c, RC)
    err_f = rel_rms(g.forces + F_N, ref.forces)
    assert 1e-5 < err_f < 4e-3
    err_e = abs(g.energy + U_N - ref.energy) / abs(ref.energy)
    assert err_e < 4e-3


# ---- ik-differentiation (App. C, eq. rhodiagforce) -------------------------
def test_ik_forces_conserve_momentum(water_small):
    """ik-differentiation conserves momentum: the net force is zero to rounding
    (analytic differentiation does not, see above)."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid_ik(h, r, q, prm)
    frms = np.sqrt(np.mean(np.sum(g.forces ** 2, axis=1)))
    assert np.linalg.norm(g.forces.sum(axis=0)) < 1e-12 * len(q) * frms


def test_ik_forces_converge_to_direct(sysA):
    """Refining window and grid drives the ik forces to the direct-sum Fourier
    forces (structure factors, no grid): pins the sign, the i k factor, the
    triclinic k vectors and the plain-window gather."""
    h, r, q, _ = sysA
    c = c_from_tol(1e-6)
    _, _, F_F = esp_direct.fourier_space(h, r, q, c, RC)
    prm = _grid_params(h, c, c_from_tol(1e-13), 16, 2.0)
    g = esp_grid.esp_grid_ik(h, r, q, prm)
    assert rel_rms(g.forces, F_F) < 1e-10


def test_ik_and_analytic_forces_agree_to_discretisation_error(water_small):
    """At working parameters both force options carry only the discretisation
    error against the direct-sum Fourier forces at the same c (ik the smaller
    one here), they are genuinely different, and energy and virial agree."""
    h, r, q, prm = water_small
    _, _, F_F = esp_direct.fourier_space(h, r, q, prm.c_split, RC)
    a = esp_grid.esp_grid(h, r, q, prm)
    b = esp_grid.esp_grid_ik(h, r, q, prm)
    assert a.energy == b.energy
    assert np.array_equal(a.virial, b.virial)
    e_ad, e_ik = rel_rms(a.forces, F_F), rel_rms(b.forces, F_F)
    assert e_ad < 3e-3 and e_ik < 3e-3
    assert 1e-9 < rel_rms(b.forces, a.forces) <= e_ad + e_ik


def test_nyquist_modes_dropped_only_for_even_grids():
    m = esp_grid.nyquist_mask((4, 5, 6))
    assert m.shape == (4, 5, 6)
    assert not m[2].any() and not m[:, :, 3].any()
    assert m.sum() == 3 * 5 * 5


# ---- per-particle (local) virial (Sec. 4.4, eq. rhodiag, eq. PinsFind) ------
def test_direct_local_virial_adds_up(sysA):
    h, r, q, _ = sysA
    c = c_from_tol(1e-6)
    _, W_F, _ = esp_direct.fourier_space(h, r, q, c, RC, forces=False)
    Wi = esp_direct.fourier_local_virial(h, r, q, c, RC)
    assert np.max(np.abs(Wi.sum(axis=0) - W_F)) < 1e-12 * np.max(np.abs(W_F))
    assert np.array_equal(Wi, np.transpose(Wi, (0, 2, 1)))


def test_grid_local_virial_adds_up(water_small):
    """The shares add up to the gridded Fourier virial (no background term for
    a neutral system) to rounding."""
    h, r, q, prm = water_small
    g = esp_grid.esp_grid(h, r, q, prm, forces=False)
    Wi = esp_grid.local_virial(h, r, q, prm)
    assert np.max(np.abs(Wi.sum(axis=0) - g.virial)) < 1e-12 * np.max(np.abs(g.virial))


def test_grid_local_virial_converges_to_direct(sysA):
    """Refining window and grid drives each particle's share to the explicit
    Fourier-sum share (pins P_hat per component, the deconvolution and the
    q_i / 2V factor particle by particle)."""
    h, r, q, _ = sysA
    c = c_from_tol(1e-6)
    ref = esp_direct.fourier_local_virial(h, r, q, c, RC)
    prm = _grid_params(h, c, c_from_tol(1e-13), 16, 2.0)
    Wi = esp_grid.local_virial(h, r, q, prm)
    assert np.max(np.abs(Wi - ref)) < 1e-10 * np.max(np.abs(ref))
