"""GPU edge cases through the C ABI: a single charge, a net charge, positions
outside the cell, non-finite input, empty and overfull tiles, box updates,
and the LDS limit."""
import numpy as np
import pytest

from gpu_util import as_inputs, oracle, paper_params, parity, parity_vs_oracle, stencil_ties, ties_of
from paper_2601_00161_amd import esp, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def explicit(prm):
    return dict(c_split=prm["c_split"], c_spread=prm["c_spread"], P=prm["P"], M=tuple(prm["M"]), rc=prm["rc"])


def run(h, r, q, prm, precision, **kw):
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    kw.setdefault("window_tol", 2e-8 if precision == "fp32" else 1e-13)
    plan = esp.Plan(h, len(q), 1e-4, precision=precision, **explicit(prm), **kw)
    xyz = torch.from_numpy(r_).to(DEV)
    qq = torch.from_numpy(q_).to(DEV)
    f, out = plan.forces(xyz, qq)
    st = plan.check()
    res = f.double().cpu().numpy(), out.cpu().numpy(), st, plan.params
    plan.close()
    return res, r64, q64


def check(label, h, res, r64, q64, prm, precision, force_abs=None):
    (f, out, st, _), ref = res, oracle(h, r64, q64, prm)
    assert st == esp.ESP_OK
    parity_vs_oracle(label, out, ref, f=f if force_abs is None else None, precision=precision,
                     ties=ties_of(h, r64, prm))
    if force_abs is not None:
        assert np.max(np.abs(f - ref.forces)) < force_abs
    return ref


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_single_charge(precision):
    """n = 1: a net charge with its neutralising background (eq. Corr)."""
    h = np.diag([2.0, 2.3, 2.1])
    r = np.array([[0.3, 1.7, 0.9]])
    q = np.array([1.0])
    prm = paper_params(h, 1e-5)
    res, r64, q64 = run(h, r, q, prm, precision)
    # the gridded force on a lone charge is only the small grid self-force;
    # compare absolutely on the natural scale q^2 / L^2 ~ 0.2
    check("single_charge", h, res, r64, q64, prm, precision, force_abs=2e-5 if precision == "fp32" else 1e-9)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_net_charge(precision):
    h, r, q = synth.random_neutral(600, np.array([[2.6, 0.3, 0.0], [0.0, 2.4, 0.2], [0.0, 0.0, 2.5]]), seed=3)
    q = q + 0.01                       # Q = 6 e
    prm = paper_params(h, 1e-5, coupling="flex")
    res, r64, q64 = run(h, r, q, prm, precision)
    check("net_charge", h, res, r64, q64, prm, precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_positions_outside_the_cell_are_wrapped(precision):
    """Positions shifted by integer combinations of the cell vectors (negative
    coordinates included) match the oracle on the same shifted inputs, and the
    unshifted results up to the rounding of the shifted inputs."""
    h, r, q = synth.water(300, np.array([[2.4, 0.2, -0.1], [0.0, 2.5, 0.3], [0.0, 0.0, 2.3]]), seed=5)
    prm = paper_params(h, 1e-5)
    shift = np.random.default_rng(1).integers(-3, 4, size=(len(q), 3)) @ h.T
    res0, _, _ = run(h, r, q, prm, precision)
    res1, r64, q64 = run(h, r + shift, q, prm, precision)
    check("wrapped", h, res1, r64, q64, prm, precision)
    # unshifted vs shifted: the shifted inputs are rounded differently (in FP32
    # an ulp of a coordinate up to ~10 nm, ~5e-7 nm), which moves particles and
    # so changes results by that much: measured virial component 2.2e-5,
    # per-particle force 1.3e-5 (FP64 1e-13).  Input rounding, not arithmetic.
    loose = 1e-4 if precision == "fp32" else 1e-10
    ties = stencil_ties(h, r.astype(np.float64), prm["M"], prm["P"], eps=1e-5)
    parity("wrapped_vs_unshifted", res1[1], res0[1][0], res0[1][1:], res1[0], res0[0], precision,
           bars=dict(energy=loose, trace=loose, virial=loose, f_rms=loose, f_max=loose), ties=ties)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_nonfinite_input_is_flagged(precision):
    """A non-finite position or charge is reported by esp_check (ESP_ENONFINITE)
    and the particle is treated as uncharged."""
    h, r, q = synth.water(200, synth.cubic(2.2), seed=6)
    prm = paper_params(h, 1e-4)
    r_bad = r.copy()
    r_bad[17, 1] = np.nan
    q_bad = q.copy()
    q_bad[40] = np.inf
    r_, q_, _, _ = as_inputs(r_bad, q_bad, precision)
    kw = {"window_tol": 1e-13 if precision == "fp64" else 2e-8}
    plan = esp.Plan(h, len(q), 1e-4, precision=precision, **explicit(prm), **kw)
    f, out = plan.forces(torch.from_numpy(r_).to(DEV), torch.from_numpy(q_).to(DEV))
    with pytest.raises(esp.EspError) as ei:
        plan.check()
    assert ei.value.status == esp.ESP_ENONFINITE
    assert plan.check() == esp.ESP_OK                      # the flag was cleared
    q_ref = q.copy()
    q_ref[[17, 40]] = 0.0
    r_ref = r.copy()
    r_ref[17] = 0.0
    _, _, r64, q64 = as_inputs(r_ref, q_ref, precision)
    ref = oracle(h, r64, q64, prm)
    out = out.cpu().numpy()
    f = f.double().cpu().numpy()
    keep = np.ones(len(q), bool)
    keep[[17, 40]] = False
    parity("nonfinite", out, ref.energy, ref.virial, f[keep], ref.forces[keep], precision,
           ties=ties_of(h, r64, prm)[keep])
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("layout", ["clustered", "one_tile"])
def test_empty_and_crowded_tiles(layout, precision):
    """Most tiles empty: all charges in one corner region, or inside a single tile."""
    h = synth.cubic(3.0)
    rng = np.random.default_rng(7)
    n = 400
    span = 0.6 if layout == "clustered" else 0.12
    r = rng.random((n, 3)) * span + 0.05
    q = rng.uniform(-1, 1, n)
    q -= q.mean()
    prm = paper_params(h, 1e-5)
    res, r64, q64 = run(h, r, q, prm, precision)
    check(f"tiles_{layout}", h, res, r64, q64, prm, precision)


def test_set_box_equals_a_new_plan():
    """esp_set_box(h2) on a plan made for h1 gives what a plan made for h2 with
    the same parameters gives (grid along the new cell vectors)."""
    h1 = np.array([[3.0, 0.2, 0.1], [0.0, 2.9, -0.2], [0.0, 0.0, 3.1]])
    h2 = h1 @ np.array([[1.01, 0.004, 0.0], [0.0, 0.995, 0.003], [0.0, 0.0, 1.007]])
    _, r, q = synth.water(400, h1, seed=8)
    prm = paper_params(h1, 1e-5, coupling="flex")
    r_, q_, _, _ = as_inputs(r, q, "fp32")
    xyz, qq = torch.from_numpy(r_).to(DEV), torch.from_numpy(q_).to(DEV)
    a = esp.Plan(h1, len(q), 1e-5, **explicit(prm))
    assert a.set_box(h2) in (esp.ESP_OK, esp.ESP_WARN_REPLAN)
    fa, oa = a.forces(xyz, qq)
    b = esp.Plan(h2, len(q), 1e-5, **explicit(prm))
    fb, ob = b.forces(xyz, qq)
    ob = ob.cpu().numpy()
    parity("set_box_vs_new_plan", oa.cpu().numpy(), ob[0], ob[1:], fa.double().cpu().numpy(),
           fb.double().cpu().numpy(), "fp32")
    a.close()
    b.close()


def test_grid_beyond_lds_is_rejected():
    """A z column too long for one workgroup's LDS is an error at plan time
    (FP64, 12,000 points), not a failed launch.  (Planes too large for LDS
    take the split x / y passes instead; see test_gpu_fft_split.py.)"""
    h = np.diag([25.0, 25.0, 20.0])
    with pytest.raises(esp.EspError) as ei:
        esp.Plan(h, 1000, 1e-5, precision="fp64", c_split=14.0, P=6, M=(8, 8, 12000))
    assert ei.value.status == esp.ESP_EINVAL
