"""GPU parity: each step of the HIP path against the CPU oracle (element by
element where the step has an elementwise result), through the C ABI.

Inputs are seeded synthetic systems; the oracle receives the same FP32 (or
FP64) inputs converted exactly to FP64 and the same explicit parameters.
"""
import numpy as np
import pytest

from gpu_util import BARS, as_inputs, oracle, paper_params, parity, parity_vs_oracle, rel_rms, ties_of
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
    # window polynomials fitted far below the parity bars (FP32: the tightest
    # fit the FP32 path takes; FP64: 1e-13), so that what is compared is the
    # arithmetic of the path, not the fit tolerance a plan is allowed to use
    extra.setdefault("window_tol", 2e-8 if precision == "fp32" else 1e-13)
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
    # P = 8 (tol 1e-7) on small tiles: few particles per tile and chunk
    h, r, q = synth.water(600, synth.cubic(2.8), config=1, seed=15)
    out.append(("water_P8_tol1e-7", h, r, q, paper_params(h, 1e-7)))
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


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def host_tile_keys(hinv, r_, M, P, T, precision):
    """A1 on the host, operation for operation as the library defines it, for a
    bit-exact comparison of the tile keys.
    FP32: s_d = (h^-1 r)_d in float-float arithmetic (h^-1 as the float pair
    hi + lo, products split exactly, error terms summed in float), wrapped to
    [0, 1) and taken as 32-bit fixed point S = floor(frac(s) 2^32); then
    U = M S, g0 = ceil(U / 2^32 - P/2) in integer arithmetic, wrapped into
    [0, M).  FP64: s = (h00 x + h01 y) + h02 z (plain products and sums),
    s - floor(s), u = s M, g0 = ceil(u - P/2).  Key = tile of g0."""
    n = r_.shape[0]
    g = np.empty((n, 3), np.int64)
    if precision == "fp32":
        f32 = np.float32
        hi = hinv.astype(f32)
        lo = (hinv - hi.astype(np.float64)).astype(f32)
        x = r_.astype(f32)
        two32 = f32(4294967296.0)
        for k in range(3):
            sh = np.zeros(n, f32)
            sl = np.zeros(n, f32)
            for j in range(3):
                h = hi[3 * k + j]
                p = h * x[:, j]
                # the exact product error, as fmaf(h, x, -p) gives it
                pe = (np.float64(h) * x[:, j].astype(np.float64) - p.astype(np.float64)).astype(f32)
                sh, e = _two_sum(sh, p)
                sl = sl + ((e + pe) + lo[3 * k + j] * x[:, j])
            fh, e2 = _two_sum(sh, -np.floor(sh))
            sl = sl + e2
            xh = fh * two32
            ih = np.floor(xh)
            t = (xh - ih) + sl * two32
            S = (ih.astype(np.int64) + np.floor(t).astype(np.int64)) & 0xFFFFFFFF
            U = S * int(M[k])
            g0 = (U - (int(P) << 31) + 0xFFFFFFFF) >> 32
            g[:, k] = np.where(g0 < 0, g0 + M[k], g0)
    else:
        x = r_.astype(np.float64)
        for k in range(3):
            s = (hinv[3 * k] * x[:, 0] + hinv[3 * k + 1] * x[:, 1]) + hinv[3 * k + 2] * x[:, 2]
            s = s - np.floor(s)
            s = np.where(s < 1.0, s, 0.0)
            g0 = np.ceil(s * float(M[k]) - 0.5 * P).astype(np.int64)
            g[:, k] = np.where(g0 < 0, g0 + M[k], np.where(g0 >= M[k], g0 - M[k], g0))
    nt = [(M[d] + T[d] - 1) // T[d] for d in range(3)]
    return ((g[:, 2] // T[2]) * nt[1] + g[:, 1] // T[1]) * nt[0] + g[:, 0] // T[0]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_sort_keys_bit_exact(case, precision, dev):
    """A1: the permutation is a permutation, the tile offsets are exactly the
    prefix sums of the host's per-tile counts, and every particle sits in the
    tile the host computes from the same arithmetic (no tolerance, no
    exemption for stencil ties).  Positions near cell faces and exact grid
    ties are added to each system."""
    name, h, r, q, prm = case
    r = np.array(r, np.float64)
    # particles placed exactly on grid planes (u - P/2 an integer) and on the cell faces
    M0 = np.array(prm["M"], np.float64)
    k = min(8, len(q) // 4)
    s_tie = (np.arange(k)[:, None] % M0[None, :] + (prm["P"] % 2) * 0.5) / M0[None, :]
    r[:k] = s_tie @ h.T
    r[k:2 * k] = np.array([0.0, 1.0, -1e-7])[np.arange(k) % 3][:, None] * h[:, np.arange(k) % 3].T
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision)
    perm, off = plan.stage_sort(to_dev(r_, dev), to_dev(q_, dev))
    perm, off = perm.cpu().numpy(), off.cpu().numpy()
    n = len(q)
    assert np.array_equal(np.sort(perm), np.arange(n))
    key = host_tile_keys(np.array(plan.params["hinv"]), r_, plan.params["M"], prm["P"], plan.params["tile"],
                         precision)
    counts = np.bincount(key, minlength=plan.params["ntiles"])
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(counts)]))
    tile_of_pos = np.searchsorted(off, np.arange(n), side="right") - 1
    got = np.empty(n, dtype=np.int64)
    got[perm] = tile_of_pos
    assert np.array_equal(got, key), f"{int(np.sum(got != key))} particles in a different tile than the host's"
    plan.close()


@pytest.mark.parametrize("tile, lds", [(4, 1), (3, 0)], ids=["5832_tiles_lds_histogram", "13824_tiles_global_counters"])
def test_sort_keys_bit_exact_many_tiles(tile, lds, dev):
    """A1 with thousands of tiles: binning workgroups take 1,024 particles
    (4 per thread) and reserve their tile ranges with one global atomic per
    occupied tile (LDS histogram), or, beyond 8,192 tiles, count straight into
    global counters; keys and offsets still match the host bit for bit, and
    the forces match a plan with the default tiles."""
    h, r, q = synth.water(60000, synth.cubic(12.2), config=1, seed=17)
    r_, q_, r64, q64 = as_inputs(r, q, "fp32")
    from paper_2601_00161_amd.esp import Plan
    plan = Plan(h, len(q), 1e-5, tile=tile)
    prm = plan.params
    print(f"many-tiles sort: n={len(q)} M={prm['M']} tile={prm['tile']} ntiles={prm['ntiles']}", flush=True)
    assert prm["ntiles"] >= 2048 and (prm["ntiles"] <= 8192) == bool(lds)
    x, c = to_dev(r_, dev), to_dev(q_, dev)
    perm, off = plan.stage_sort(x, c)
    perm, off = perm.cpu().numpy(), off.cpu().numpy()
    n = len(q)
    assert np.array_equal(np.sort(perm), np.arange(n))
    key = host_tile_keys(np.array(prm["hinv"]), r_, prm["M"], prm["P"], prm["tile"], "fp32")
    counts = np.bincount(key, minlength=prm["ntiles"])
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(counts)]))
    tile_of_pos = np.searchsorted(off, np.arange(n), side="right") - 1
    got = np.empty(n, dtype=np.int64)
    got[perm] = tile_of_pos
    assert np.array_equal(got, key)
    f1, o1 = plan.forces(x, c)
    ref = Plan(h, n, 1e-5)
    f0, o0 = ref.forces(x, c)
    torch.cuda.synchronize()
    plan.check()
    parity(f"many_tiles_T{tile}", o1.cpu().numpy(), o0[0].item(), o0[1:].cpu().numpy(),
           f1.double().cpu().numpy(), f0.double().cpu().numpy(), "fp32")
    plan.close()
    ref.close()


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
    parity_vs_oracle(f"energy_virial/{name}", out, ref, precision=precision)
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
    parity_vs_oracle(f"forces/{name}/{accum}", out, ref, f=f, precision=precision, ties=ties_of(h, r64, prm))
    # the force path's energy and virial are those of the single-FFT path, up
    # to the order in which the spreading adds its tiles into the grid
    assert np.max(np.abs(out - out_ev)) <= (1e-6 if precision == "fp32" else 1e-12) * np.max(np.abs(out_ev))
    plan.close()


@pytest.mark.parametrize("gather", ["particle", "tile", "lane"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=IDS)
def test_forces_every_gather_variant(case, precision, gather, dev):
    """A6 with each gather forced: per particle from L2, tile-staged with a
    group of lanes per particle, tile-staged with one lane per particle."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    plan = make_plan(h, len(q), prm, precision, gather=gather)
    assert plan.params["gather_tiled"] == (0 if gather == "particle" else 1)
    assert plan.params["gather_lane"] == (1 if gather == "lane" else 0)
    f, out = plan.forces(to_dev(r_, dev), to_dev(q_, dev))
    assert plan.check() == 0
    ref = oracle(h, r64, q64, prm)
    parity_vs_oracle(f"gather_{gather}/{name}", out.cpu().numpy(), ref, f=f.cpu().numpy().astype(np.float64),
                     precision=precision, ties=ties_of(h, r64, prm))
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
    parity_vs_oracle(f"forces_ik/{name}", out, ref, f=f, precision=precision, ties=ties_of(h, r64, prm))
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
    # each of the six components over all particles: relative RMS, and the
    # largest per-particle difference against the component's RMS
    keep = ~ties_of(h, r64, prm)
    for c in range(6):
        e_rms = rel_rms(w6[keep, c], ref6[keep, c])
        e_max = np.max(np.abs(w6[keep, c] - ref6[keep, c])) / np.sqrt(np.mean(ref6[keep, c] ** 2))
        print(f"PARITY local_virial/{name}[{c}] {precision} rms={e_rms:.2e} max={e_max:.2e}", flush=True)
        assert e_rms < BARS[precision]["f_rms"] and e_max < BARS[precision]["f_max"], (c, e_rms, e_max)
    total = w6.sum(axis=0)
    assert np.max(np.abs(total - out[1:])) <= (1e-6 if precision == "fp32" else 1e-11) * np.max(np.abs(out[1:]))
    plan.close()
