"""The xy transforms as separate x and y passes (planes beyond one
workgroup's LDS, or forced with esp_opts.fft_split): the forward transform
against numpy.fft.rfftn, every force/virial path against the one-pass
transform and the oracle, and an FP64 plan on the 135 x 135 x 108 grid that
needs the split passes."""
import numpy as np
import pytest

from gpu_util import as_inputs, oracle, paper_params, parity, parity_vs_oracle, rel_rms, ties_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_00161_amd import esp, synth  # noqa: E402

DEV = "cuda:0"


def plan_for(h, n, prm, precision, **kw):
    kw.setdefault("window_tol", 2e-8 if precision == "fp32" else 1e-13)
    return esp.Plan(h, n, 1e-4, precision=precision, c_split=prm["c_split"], c_spread=prm["c_spread"],
                    P=prm["P"], M=tuple(prm["M"]), rc=prm["rc"], **kw)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("M", [(15, 15, 15), (36, 36, 36), (48, 50, 54), (16, 9, 25), (20, 27, 8), (4, 6, 5),
                               (135, 45, 9)])
def test_split_fft_against_numpy(M, precision):
    """A3 with the split passes: odd row counts (a last row without a partner),
    ragged last groups of row pairs and of columns."""
    h = np.diag([4.0, 4.0, 4.0])
    prm = dict(c_split=10.0, c_spread=10.0, P=min(4, min(M)), M=M, rc=0.9)
    plan = plan_for(h, 8, prm, precision, fft_split=True)
    assert plan.params["fft_split"] == 1
    rng = np.random.default_rng(sum(M) + 1)
    dt = np.float32 if precision == "fp32" else np.float64
    grid = rng.normal(size=(M[2], M[1], M[0])).astype(dt)
    spec = plan.stage_fft(torch.from_numpy(grid).to(DEV)).cpu().numpy()
    ref = np.fft.rfftn(grid.astype(np.float64))
    err = np.max(np.abs(spec - ref)) / np.max(np.abs(ref))
    assert err < (2e-6 if precision == "fp32" else 1e-13), err
    plan.close()


def _systems():
    tri = np.array([[3.1, 0.4, 0.3], [0.0, 2.9, -0.2], [0.0, 0.0, 3.3]])
    out = []
    h, r, q = synth.water(400, tri, config=1, seed=31)
    out.append(("water_triclinic_flex", h, r, q, paper_params(h, 1e-5, coupling="flex")))
    h, r, q = synth.water(200, np.diag([2.5, 3.0, 2.0]), config=1, seed=32)
    out.append(("orthorhombic_oddgrid_P7", h, r, q, dict(paper_params(h, 1e-6), M=(27, 25, 25))))
    return out


SYSTEMS = _systems()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("case", SYSTEMS, ids=[c[0] for c in SYSTEMS])
def test_split_paths_match_one_pass_and_oracle(case, precision):
    """Energy/virial, AD forces, ik forces and per-particle virials with the
    split passes equal the one-pass results and the oracle's."""
    name, h, r, q, prm = case
    r_, q_, r64, q64 = as_inputs(r, q, precision)
    xyz, qq = torch.from_numpy(r_).to(DEV), torch.from_numpy(q_).to(DEV)
    same = 2e-6 if precision == "fp32" else 1e-12
    ref = oracle(h, r64, q64, prm)
    for kw in ({}, {"force": "ik"}, {"local_virial": True}):
        a = plan_for(h, len(q), prm, precision, fft_split=True, **kw)
        b = plan_for(h, len(q), prm, precision, **kw)
        assert a.params["fft_split"] == 1 and b.params["fft_split"] == 0
        fa, oa = a.forces(xyz, qq)
        fb, ob = b.forces(xyz, qq)
        ea = a.energy_virial(xyz, qq).cpu().numpy()
        fa, fb = fa.double().cpu().numpy(), fb.double().cpu().numpy()
        oa, ob = oa.cpu().numpy(), ob.cpu().numpy()
        parity(f"split_vs_one_pass/{name}/{kw}", oa, ob[0], ob[1:], fa, fb, precision,
               bars=dict(energy=same, virial=same, f_rms=same, f_max=10 * same))
        parity_vs_oracle(f"split/{name}/{kw}", ea, ref, f=fa if not kw else None, precision=precision,
                         ties=ties_of(h, r64, prm))
        if kw.get("local_virial"):
            wa, _ = a.local_virial(xyz, qq)
            wb, _ = b.local_virial(xyz, qq)
            wa, wb = wa.double().cpu().numpy(), wb.double().cpu().numpy()
            assert rel_rms(wa, wb) < same
        assert a.check() == esp.ESP_OK
        a.close()
        b.close()


def test_fp64_plan_on_a_plane_beyond_lds():
    """The 25 x 25 x 20 nm slab grid (135 x 135 x 108) in FP64: its complex
    plane does not fit one workgroup's LDS, so the plan takes the split
    passes; energy, virial and forces against the oracle."""
    h = np.diag([25.0, 25.0, 20.0])
    rng = np.random.default_rng(33)
    n = 2000
    r = rng.uniform(0, 1, size=(n, 3)) * np.array([25.0, 25.0, 20.0])
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    prm = dict(c_split=14.0, c_spread=14.0, P=6, M=(135, 135, 108), rc=0.9)
    plan = plan_for(h, n, prm, "fp64")
    assert plan.params["fft_split"] == 1
    f, out = plan.forces(torch.from_numpy(r).to(DEV), torch.from_numpy(q).to(DEV))
    ref = oracle(h, r, q, prm)
    out = out.cpu().numpy()
    parity_vs_oracle("split/slab_plane_fp64", out, ref, f=f.cpu().numpy(), precision="fp64",
                     ties=ties_of(h, r, prm))
    plan.close()
