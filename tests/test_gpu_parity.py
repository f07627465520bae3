"""GPU parity: each step of the HIP path against the CPU oracle (element by
element where the step has an elementwise result), through the C ABI.

Inputs are seeded synthetic systems; the oracle receives the same FP32 (or
FP64) inputs converted exactly to FP64 and the same explicit parameters.
"""
import numpy as np
import pytest

from gpu_util import TOL, as_inputs, oracle, paper_params, rel_rms, tensor_rel, w6
from paper_2601_00161_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def make_plan(h, n, prm, precision, **kw):
    from paper_2601_00161_amd.esp import Plan
    extra = dict(kw)
    if precision == "fp64":
        extra.setdefault("window_tol", 1e-13)
    return Plan(h, n, 1e-4, precision=precision, c_split=prm["c_split"], c_spread=prm["c_spread"],
                P=prm["P"], M=prm["M"], rc=prm["rc"], **extra)


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


TRICLINIC = np.array([[3.1, 0.4, 0.3], [0.0, 2.9, -0.2], [0.0, 0.0, 3.3]])


def systems():
    """(name, h, r, q, prm): small cases spanning several tiles and ragged tails."""
    out = []
    h, r, q = synth.water(300, synth.cubic(2.2), config=1, seed=11)
    out.append(("water_cubic_tol1e-4", h, r, q, paper_params(h, 1e-4)))
    h, r, q = synth.water(400, TRICLINIC, config=1, seed=12)
    out.append(("water_triclinic_flex", h, r, q, paper_params(h, 1e-5, coupling="flex")))
    h, r, q = synth.ionic(40, h=np.array([[3.2, 0.5, 0.3], [0.0, 3.0, 0.2], [0.0, 0.0, 3.1]]), seed=3)
    out.append(("ionic_triclinic_P4", h, r, q, dict(paper_params(h, 1e-3), P=4)))
    h, r, q = synth.water(200, np.diag([2.5, 3.0, 2.0]), config=1, seed=13)
    out.append(("orthorhombic_oddgrid_P7", h, r, q, dict(paper_params(h, 1e-6), M=(27, 30, 25))))
    # dense tiles (coarse grid, many particles per tile): the tile-staged gather
    # and the binning with tile-counter copies
    h, r, q = synth.water(7200, synth.cubic(6.0), config=1, seed=14)
    out.append(("water_dense_tiles_tol1e-3", h, r, q, paper_params(h, 1e-3)))
    return out


def test_paths_are_covered(dev):
    """The systems above exercise both gather variants and both binning modes."""
    modes = set()
    for name, h, r, q, prm in SYSTEMS:
        plan = make_plan(h, len(q), prm, "fp32")
        modes.add(("tiled", plan.params["gather_tiled"]))
        modes.add(("copies", plan.params["counter_copies"] > 1))
        plan.close()
    assert {("tiled", 0), ("tiled", 1), ("copies", False), ("copies", True)} <= modes, modes


SYSTEMS = systems()
IDS = [s[0] for s in SYSTEMS]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_sort_is_a_valid_binning(case, precision, dev):
    """A1: the permutation is a permutation, tile offsets partition it, and each
    particle sits in the tile of its stencil base g0 = ceil(u - P/2) (checked on
    the host from FP64 reduced coordinates; near-tie cases may go either way)."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision)
    perm, off = plan.stage_sort(to_dev(r_, dev), to_dev(q_, dev))
    perm, off = perm.cpu().numpy(), off.cpu().numpy()
    n = len(q)
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    T = plan.params["tile"]
    M = np.array(plan.params["M"])
    s = np.linalg.solve(h, r64.T).T
    s -= np.floor(s)
    u = s * M
    g0 = np.ceil(u - prm["P"] / 2.0)
    frac = np.abs((u - prm["P"] / 2.0) - np.round(u - prm["P"] / 2.0))
    g0 = g0.astype(np.int64) % M
    nt = [(M[d] + T[d] - 1) // T[d] for d in range(3)]
    key = ((g0[:, 2] // T[2]) * nt[1] + g0[:, 1] // T[1]) * nt[0] + g0[:, 0] // T[0]
    tile_of_pos = np.searchsorted(off, np.arange(n), side="right") - 1
    got = np.empty(n, dtype=np.int64)
    got[perm] = tile_of_pos
    ok = (got == key) | np.any(frac < 1e-6, axis=1)
    assert ok.all(), f"{(~ok).sum()} particles in the wrong tile"
    plan.close()


def test_spread_accumulator_rule(dev):
    """The automatic choice takes 64-bit fixed point for FP32 plans, and for
    FP64 plans exactly when there are at least 512 tiles holding at least
    128 particles on average; explicit choices are kept."""
    for name, h, r, q, prm in SYSTEMS:
        for tile in (0, 8):
            plan = make_plan(h, len(q), prm, "fp32", tile=tile)
            assert plan.params["spread_fixed"] == 1, (name, tile)
            plan.close()
            plan = make_plan(h, len(q), prm, "fp64", tile=tile)
            nt = plan.params["ntiles"]
            want = nt >= 512 and len(q) >= 128 * nt
            assert plan.params["spread_fixed"] == int(want), (name, tile)
            plan.close()
        for precision in ("fp32", "fp64"):
            for accum, want in (("fixed", 1), ("fp64", 0)):
                plan = make_plan(h, len(q), prm, precision, spread_accum=accum)
                assert plan.params["spread_fixed"] == want
                plan.close()


@pytest.mark.parametrize("accum", ["fixed", "fp64"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_spread_grid(case, precision, accum, dev):
    """A2: the charge grid equals the oracle's Step-1 grid element by element,
    with either LDS accumulator."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, spread_accum=accum)
    g = plan.stage_spread(to_dev(r_, dev), to_dev(q_, dev)).cpu().numpy().astype(np.float64)
    ref = oracle(h, r64, q64, prm, forces=False).rho_grid.transpose(2, 1, 0)
    # scale: the largest cell of the same grid spread with |q| (no cancellation).
    # The window fit error is absolute (<= window_tol psi(0) per weight), so the
    # bar is global: FP32 rounding of weights and products (a few 2^-24), FP64
    # the 1e-13 window fit.
    scale = np.max(oracle(h, r64, np.abs(q64), prm, forces=False).rho_grid)
    bar = 1e-6 if precision == "fp32" else 1e-12
    err = np.max(np.abs(g - ref)) / scale
    assert err < bar, err
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("M", [(15, 15, 15), (36, 36, 36), (48, 50, 54), (16, 9, 25), (20, 27, 8), (4, 6, 5)])
def test_fft_against_numpy(M, precision, dev):
    """A3: forward real-to-complex 3D FFT equals numpy.fft.rfftn on the same grid."""
    h = np.diag([4.0, 4.0, 4.0])
    prm = dict(c_split=10.0, c_spread=10.0, P=min(4, min(M)), M=M, rc=0.9)
    plan = make_plan(h, 8, prm, precision)
    rng = np.random.default_rng(sum(M))
    dt = np.float32 if precision == "fp32" else np.float64
    grid = rng.normal(size=(M[2], M[1], M[0])).astype(dt)
    spec = plan.stage_fft(to_dev(grid, dev)).cpu().numpy()
    ref = np.fft.rfftn(grid.astype(np.float64))
    err = np.max(np.abs(spec - ref)) / np.max(np.abs(ref))
    assert err < (2e-6 if precision == "fp32" else 1e-13), err
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("qscale", [1e-12, 1e12])
def test_fixed_point_spread_follows_the_charge_scale(qscale, precision, dev):
    """The fixed-point scale is chosen per tile from its charges: charges
    multiplied by 1e-12 or 1e12 give the same grid times that factor (the
    scale is a power of two, so up to the rounding of the factor itself), and
    uncharged particles give an exactly zero grid."""
    name, h, r, q, prm = SYSTEMS[0]
    r_, q_, _, _ = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, spread_accum="fixed")
    g1 = plan.stage_spread(to_dev(r_, dev), to_dev(q_, dev)).cpu().numpy().astype(np.float64)
    qs = (q_.astype(np.float64) * qscale).astype(q_.dtype)
    g2 = plan.stage_spread(to_dev(r_, dev), to_dev(qs, dev)).cpu().numpy().astype(np.float64)
    g0 = plan.stage_spread(to_dev(r_, dev), to_dev(np.zeros_like(q_), dev)).cpu().numpy()
    plan.close()
    bar = 1e-6 if precision == "fp32" else 1e-12
    assert np.all(np.isfinite(g2))
    assert np.max(np.abs(g2 / qscale - g1)) <= bar * np.max(np.abs(g1))
    assert not np.any(g0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_energy_virial(case, precision, dev):
    """A4 + A7: energy and the six virial components from the single-FFT path."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision)
    out = plan.energy_virial(to_dev(r_, dev), to_dev(q_, dev)).cpu().numpy()
    ref = oracle(h, r64, q64, prm, forces=False)
    assert abs(out[0] - ref.energy) / abs(ref.energy) < TOL[precision]
    assert tensor_rel(out, ref.virial) < TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_potential_grid(case, precision, dev):
    """A5: the potential grid phi (inverse FFT of F_hat rho_hat / (V W_hat^2))."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision)
    phi = plan.stage_potential(to_dev(r_, dev), to_dev(q_, dev)).cpu().numpy().astype(np.float64)
    ref = oracle(h, r64, q64, prm).phi_grid.transpose(2, 1, 0)
    err = np.max(np.abs(phi - ref)) / np.max(np.abs(ref))
    assert err < (1e-5 if precision == "fp32" else 1e-10), err
    plan.close()


@pytest.mark.parametrize("accum", ["fixed", "fp64"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_forces(case, precision, accum, dev):
    """A6: forces by analytic differentiation; E and W from the force path equal
    those of the single-FFT path (either LDS accumulator of the spreading)."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, spread_accum=accum)
    xyz, qq = to_dev(r_, dev), to_dev(q_, dev)
    f, out = plan.forces(xyz, qq)
    f = f.cpu().numpy().astype(np.float64)
    out = out.cpu().numpy()
    out_ev = plan.energy_virial(xyz, qq).cpu().numpy()
    ref = oracle(h, r64, q64, prm)
    assert rel_rms(f, ref.forces) < TOL[precision]
    assert abs(out[0] - ref.energy) / abs(ref.energy) < TOL[precision]
    assert tensor_rel(out, ref.virial) < TOL[precision]
    assert np.max(np.abs(out - out_ev)) <= 1e-6 * np.max(np.abs(out_ev)) + 1e-12
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_forces_ik(case, precision, dev):
    """ik-differentiation (App. C, eq. rhodiagforce): forces against the oracle's
    ik forces, energy and virial unchanged, and the net force zero up to the
    rounding of the forces themselves."""
    from oracle import esp_grid
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, force="ik")
    assert plan.params["force"] == 1
    f, out = plan.forces(to_dev(r_, dev), to_dev(q_, dev))
    f = f.cpu().numpy().astype(np.float64)
    out = out.cpu().numpy()
    ref = esp_grid.esp_grid_ik(h, r64, q64, esp_grid.GridParams(prm["c_split"], prm["c_spread"], prm["P"],
                                                                tuple(prm["M"]), prm["rc"]))
    assert rel_rms(f, ref.forces) < TOL[precision]
    assert abs(out[0] - ref.energy) / abs(ref.energy) < TOL[precision]
    assert tensor_rel(out, ref.virial) < TOL[precision]
    fscale = np.sqrt(np.mean(np.sum(ref.forces ** 2, axis=1)))
    eps = 1e-6 if precision == "fp32" else 1e-12
    assert np.linalg.norm(f.sum(axis=0)) < eps * np.sqrt(len(q)) * fscale
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_local_virial(case, precision, dev):
    """Per-particle Fourier virial (Sec. 4.4, eq. PinsFind) against the oracle,
    and the shares adding up to the plan's virial (neutral systems)."""
    from oracle import esp_grid
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, local_virial=True)
    out7 = torch.empty(7, dtype=torch.float64, device=dev)
    w6, _ = plan.local_virial(to_dev(r_, dev), to_dev(q_, dev), out7=out7)
    w6 = w6.cpu().numpy().astype(np.float64)
    out = out7.cpu().numpy()
    ref = esp_grid.local_virial(h, r64, q64, esp_grid.GridParams(prm["c_split"], prm["c_spread"], prm["P"],
                                                                 tuple(prm["M"]), prm["rc"]))
    ref6 = np.stack([ref[:, 0, 0], ref[:, 1, 1], ref[:, 2, 2], ref[:, 0, 1], ref[:, 0, 2], ref[:, 1, 2]], axis=1)
    assert rel_rms(w6, ref6) < TOL[precision]
    total = w6.sum(axis=0)
    assert np.max(np.abs(total - out[1:])) <= (1e-6 if precision == "fp32" else 1e-11) * np.max(np.abs(out[1:]))
    plan.close()
