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
    b = esp.Plan(h, len(q), 1e-4, gather="tile")
    assert a.params["gather_tiled"] == 0 and b.params["gather_tiled"] == 1
    fa, oa = a.forces(xyz, qq)
    fb, ob = b.forces(xyz, qq)
    assert rel_rms(fb.double().cpu().numpy(), fa.double().cpu().numpy()) < 1e-6
    assert np.max(np.abs(ob.cpu().numpy() - oa.cpu().numpy())) <= 1e-6 * np.max(np.abs(oa.cpu().numpy()))
    a.close()
    b.close()
