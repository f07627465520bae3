"""The launch-shape autotuner: admissible choices, a reused JSON cache, and
tuned plans that compute the same results as the default plan."""
import json

import numpy as np
import pytest

from gpu_util import rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_00161_amd import autotune, esp, synth  # noqa: E402

DEV = "cuda:0"


def test_tuned_plan_matches_default_and_caches(tmp_path):
    h, r, q = synth.water(3000, synth.cubic(4.5), config=1, seed=9)
    xyz = torch.tensor(r, dtype=torch.float32, device=DEV)
    qq = torch.tensor(q, dtype=torch.float32, device=DEV)
    cache = str(tmp_path / "tune.json")
    plan, info = autotune.tuned_plan(h, len(q), 1e-5, xyz, qq, cache=cache)
    assert info["tile"] in autotune.TILES and info["gather"] in autotune.GATHERS
    assert info["accum"] in autotune.ACCUMS
    key = f"{info['tile']}:{info['gather']}" + (":fixed" if info["accum"] == "fixed" else "")
    assert key in info["table"]
    assert plan.params["spread_fixed"] == (1 if info["accum"] == "fixed" else 0)
    # an FP32 plan tries both accumulators for every tile and gather variant
    for k in list(info["table"]):
        if not k.endswith(":fixed"):
            assert k + ":fixed" in info["table"]
    assert plan.params["tile"][0] == min(info["tile"], plan.params["M"][0])
    assert plan.params["gather_tiled"] == (1 if info["gather"] == "tile" else 0)
    data = json.load(open(cache))
    assert info["key"] in data
    f1, o1 = plan.forces(xyz, qq)
    ref = esp.Plan(h, len(q), 1e-5)
    f0, o0 = ref.forces(xyz, qq)
    assert rel_rms(f1.double().cpu().numpy(), f0.double().cpu().numpy()) < 2e-6
    assert np.max(np.abs(o1.cpu().numpy() - o0.cpu().numpy())) <= 2e-6 * np.max(np.abs(o0.cpu().numpy()))
    # second request: served from the cache (the stored timing table is unchanged)
    plan2, info2 = autotune.tuned_plan(h, len(q), 1e-5, xyz, qq, cache=cache)
    assert info2["table"] == info["table"]
    for p in (plan, plan2, ref):
        p.close()


def test_forced_gather_variants_agree():
    h, r, q = synth.water(4000, synth.cubic(5.0), config=1, seed=10)
    xyz = torch.tensor(r, dtype=torch.float32, device=DEV)
    qq = torch.tensor(q, dtype=torch.float32, device=DEV)
    a = esp.Plan(h, len(q), 1e-4, gather="particle")
    fa, oa = a.forces(xyz, qq)
    for g in ("tile", "lane"):
        b = esp.Plan(h, len(q), 1e-4, gather=g)
        assert a.params["gather_tiled"] == 0 and b.params["gather_tiled"] == 1
        assert b.params["gather_lane"] == (1 if g == "lane" else 0)
        fb, ob = b.forces(xyz, qq)
        assert rel_rms(fb.double().cpu().numpy(), fa.double().cpu().numpy()) < 1e-6
        assert np.max(np.abs(ob.cpu().numpy() - oa.cpu().numpy())) <= 1e-6 * np.max(np.abs(oa.cpu().numpy()))
        b.close()
    a.close()


def test_tuned_batch_matches_default_batch(tmp_path):
    """The batch autotuner (tile edge per window-support group, timed on the
    batch itself) picks admissible tiles, caches its choice, and the tuned
    batch computes the default batch's results up to reassociation."""
    import gpu_util as gu
    reps = synth.replicas(n_rep=6, config=5, seed=3, n_range=(2000, 9000))
    cells = [x[0] for x in reps]
    ns = [len(x[2]) for x in reps]
    tols = [x[3] for x in reps]
    xyz = torch.tensor(np.concatenate([x[1] for x in reps]), dtype=torch.float32, device=DEV)
    qq = torch.tensor(np.concatenate([x[2] for x in reps]), dtype=torch.float32, device=DEV)
    cache = str(tmp_path / "tune.json")
    info = autotune.tune_batch(cells, ns, tols, xyz, qq, cache=cache, tiles=(4, 6, 8))
    b0 = esp.Batch(cells, ns, tols)
    Ps = sorted({p["P"] for p in b0.params})
    assert len(info["tiles"]) == len(ns)
    assert sorted(int(k) for k in info["groups"]) == Ps
    assert all(t in (0, 4, 6, 8) for t in info["tiles"])
    assert info["ms"] <= info["default_ms"]
    assert autotune.tune_batch(cells, ns, tols, xyz, qq, cache=cache, tiles=(4, 6, 8))["tiles"] == info["tiles"]
    b1 = esp.Batch(cells, ns, tols, tiles=info["tiles"])
    for b, t in zip(b1.params, info["tiles"]):
        if t:
            assert b["tile"][0] == min(t, b["M"][0])
    f0, o0 = b0.forces(xyz, qq)
    f1, o1 = b1.forces(xyz, qq)
    torch.cuda.synchronize()
    b0.check()
    b1.check()
    o0, o1 = o0.cpu().numpy(), o1.cpu().numpy()
    f0, f1 = f0.double().cpu().numpy(), f1.double().cpu().numpy()
    for r in range(len(ns)):
        a, e = b0.offsets[r], b0.offsets[r + 1]
        gu.parity(f"tuned_batch_rep{r}", o1[r], o0[r][0], o0[r][1:], f1[a:e], f0[a:e], "fp32")
    b0.close()
    b1.close()
