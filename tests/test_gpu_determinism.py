"""Run-to-run repeatability of deterministic FP32 plans (esp_opts.deterministic).

Each tile sums its terms as integers and adds them to an int64 grid at one
scale per call, so no floating-point sum depends on the order in which
workgroups or atomics run: repeated calls on the same inputs return the same
bits (energy, virial and every force component), whether the cell sort uses
one tile counter per tile or counter copies, for single plans, batches and the
allocation-free entry point.  The default (non-deterministic) plans add tile
cells with floating-point atomics and are checked against them to the parity
bar."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import gpu_util as gu  # noqa: E402
from paper_2601_00161_amd import esp, synth  # noqa: E402

DEV = "cuda:0"


def _dev(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).to(DEV)


def _same(a, b):
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("n_mol, L, tol, opts", [
    (3000, 4.5, 1e-5, dict()),                       # one counter per tile
    (3000, 4.5, 1e-5, dict(coupling="flex", gather="particle")),
    (3000, 4.5, 1e-5, dict(fft_split=True)),         # split x / y passes read the int64 grid
    (100000, 10.0, 1e-3, dict(tile=4)),              # counter copies (nsub > 1)
])
def test_repeated_calls_return_identical_bits(n_mol, L, tol, opts):
    h, r, q = synth.water(n_mol, synth.cubic(L), config=1, seed=21)
    x, c = _dev(r), _dev(q)
    plan = esp.Plan(h, len(q), tol, deterministic=True, **opts)
    prm = plan.params
    print(f"determinism n={len(q)} tol={tol} opts={opts} tiles={prm['ntiles']} "
          f"copies={prm['counter_copies']} fixed={prm['spread_fixed']}", flush=True)
    assert prm["spread_fixed"] == 1 and prm["grid_fixed"] == 1
    if len(q) > 200000:
        assert prm["counter_copies"] > 1
    f0, o0 = plan.forces(x, c)
    e0 = plan.energy_virial(x, c)
    for _ in range(3):
        f1, o1 = plan.forces(x, c)
        assert _same(f1, f0) and _same(o1, o0)
    assert _same(plan.energy_virial(x, c), e0)
    g0 = plan.stage_spread(x, c)
    assert _same(plan.stage_spread(x, c), g0)
    torch.cuda.synchronize()
    plan.check()
    # the default plan (floating-point grid atomics) agrees to the parity bar
    ref = esp.Plan(h, len(q), tol, **opts)
    assert ref.params["grid_fixed"] == 0
    fr, orr = ref.forces(x, c)
    gu.parity(f"deterministic_vs_default_n{len(q)}", o0.cpu().numpy(), orr[0].item(), orr[1:].cpu().numpy(),
              f0.double().cpu().numpy(), fr.double().cpu().numpy(), "fp32")
    ref.close()
    plan.close()


def test_batch_and_noalloc_repeat_bit_for_bit():
    reps = synth.replicas(n_rep=5, config=5, seed=4, n_range=(2000, 9000))
    cells = [x[0] for x in reps]
    ns = [len(x[2]) for x in reps]
    tols = [x[3] for x in reps]
    xyz = _dev(np.concatenate([x[1] for x in reps]))
    qq = _dev(np.concatenate([x[2] for x in reps]))
    for graph in (False, True):
        b = esp.Batch(cells, ns, tols, graph=graph, deterministic=True)
        assert all(p["grid_fixed"] == 1 for p in b.params)
        f0, o0 = b.forces(xyz, qq)
        f0, o0 = f0.clone(), o0.clone()
        for _ in range(3):
            f1, o1 = b.forces(xyz, qq)
            assert _same(f1, f0) and _same(o1, o0)
        torch.cuda.synchronize()
        b.check()
        b.close()
    h, r, q = synth.water(2000, synth.cubic(4.0), config=1, seed=5)
    x, c = _dev(r), _dev(q)
    fa, oa = esp.forces_noalloc(h, x, c, 1e-5, deterministic=True)
    fa, oa = fa.clone(), oa.clone()
    fb, ob = esp.forces_noalloc(h, x, c, 1e-5, deterministic=True)
    assert _same(fa, fb) and _same(oa, ob)
    plan = esp.Plan(h, len(q), 1e-5, deterministic=True)
    fp, op = plan.forces(x, c)
    # the same plan built in the scratch region runs the same kernels
    assert _same(fp, fa) and _same(op, oa)
    plan.close()


def test_deterministic_batch_needs_fixed_point_tiles(capfd):
    """FP32 batches spread in fixed point whatever spread_accum says; with
    spread_accum = fp64 their plans have no int64 grid, which a deterministic
    batch refuses, while a default batch runs."""
    reps = synth.replicas(n_rep=2, config=5, seed=4, n_range=(2000, 3000))
    args = ([x[0] for x in reps], [len(x[2]) for x in reps], [x[3] for x in reps])
    b = esp.Batch(*args, spread_accum="fp64")
    assert all(p["grid_fixed"] == 0 for p in b.params)
    b.close()
    b = esp.Batch(*args, deterministic=True)
    assert all(p["grid_fixed"] == 1 for p in b.params)
    b.close()
