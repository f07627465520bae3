"""Batched evaluation of many replicas (one launch per stage) against the
single-plan path and the oracle, with and without HIP-graph replay."""
import numpy as np
import pytest

import gpu_util as gu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_00161_amd import esp, synth  # noqa: E402

DEV = "cuda:0"


def _replicas(n_rep=8, seed=0):
    reps = synth.replicas(n_rep=n_rep, config=5, seed=seed, n_range=(2000, 12000))
    cells = [h for h, _, _, _ in reps]
    pos = [p for _, p, _, _ in reps]
    qs = [q for _, _, q, _ in reps]
    tols = [t for _, _, _, t in reps]
    return cells, pos, qs, tols


def _cat(arrs, dtype):
    return torch.tensor(np.concatenate(arrs), dtype=dtype, device=DEV).contiguous()


def _close(a, b, rel):
    """Energy and each virial component within rel (components against
    max(|W_c|, FLOOR max |W_aa|)), for one or several out7 rows."""
    a = np.atleast_2d(np.asarray(a, np.float64))
    b = np.atleast_2d(np.asarray(b, np.float64))
    for x, y in zip(a, b):
        if abs(x[0] - y[0]) > rel * abs(y[0]) or np.any(gu.component_errors(x, y[1:]) > rel):
            return False
    return True


def _forces_close(f, g, rel):
    """Relative RMS within rel and the largest per-particle difference within
    10 rel of the RMS force."""
    e_rms, e_max = gu.force_errors(f, g)
    return e_rms < rel and e_max < 10 * rel


@pytest.fixture(scope="module")
def system():
    return _replicas()


def _single(cells, pos, qs, tols, r, dtype, prm=None, window_tol=0.0):
    kw = {} if prm is None else dict(c_split=prm["c_split"], P=prm["P"], M=tuple(prm["M"]))
    plan = esp.Plan(cells[r], len(qs[r]), tols[r], precision="fp32" if dtype == torch.float32 else "fp64",
                    window_tol=window_tol, **kw)
    x = torch.tensor(pos[r], dtype=dtype, device=DEV)
    q = torch.tensor(qs[r], dtype=dtype, device=DEV)
    f, o = plan.forces(x, q)
    e = plan.energy_virial(x, q)
    torch.cuda.synchronize()
    out = f.double().cpu().numpy(), o.cpu().numpy(), e.cpu().numpy()
    plan.close()
    return out


def test_batch_covers_several_supports(system):
    cells, pos, qs, tols = system
    b = esp.Batch(cells, [len(q) for q in qs], tols)
    Ps = {p["P"] for p in b.params}
    assert len(Ps) >= 2
    # one launch per stage, plus one spread / gather launch per extra (P, window degree) group
    assert b.num_launches(True) <= 7 + 2 * (len(Ps) * 3 - 1)
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_batch_matches_single_plans(system, precision):
    cells, pos, qs, tols = system
    dt = torch.float32 if precision == "fp32" else torch.float64
    b = esp.Batch(cells, [len(q) for q in qs], tols, precision=precision)
    x, q = _cat(pos, dt), _cat(qs, dt)
    f, o = b.forces(x, q)
    e = b.energy_virial(x, q)
    assert b.check() == esp.ESP_OK
    f = f.double().cpu().numpy()
    o, e = o.cpu().numpy(), e.cpu().numpy()
    rel = 2e-6 if precision == "fp32" else 1e-12
    for r in range(len(qs)):
        fs, os_, es = _single(cells, pos, qs, tols, r, dt)
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert _forces_close(f[sl], fs, rel), r
        assert _close(o[r], os_, rel), (r, o[r], os_)
        assert _close(e[r], es, rel), (r, e[r], es)
    b.close()


def test_batch_fp64_matches_oracle(system):
    cells, pos, qs, tols = system
    b = esp.Batch(cells[:3], [len(q) for q in qs[:3]], tols[:3], precision="fp64", window_tol=1e-13)
    x, q = _cat(pos[:3], torch.float64), _cat(qs[:3], torch.float64)
    f, o = b.forces(x, q)
    f = f.cpu().numpy()
    o = o.cpu().numpy()
    for r in range(3):
        ref = gu.oracle(cells[r], pos[r], qs[r], b.params[r])
        sl = slice(b.offsets[r], b.offsets[r + 1])
        gu.parity_vs_oracle(f"batch_fp64/rep{r}", o[r], ref, f=f[sl], precision="fp64",
                            ties=gu.ties_of(cells[r], pos[r], b.params[r]))
    b.close()


def test_batch_graph_replays_match_eager(system):
    cells, pos, qs, tols = system
    ns = [len(q) for q in qs]
    b = esp.Batch(cells, ns, tols, graph=True)
    x, q = _cat(pos, torch.float32), _cat(qs, torch.float32)
    f, o = b.forces(x, q)                       # eager run + recording
    torch.cuda.synchronize()
    f0, o0 = f.double().cpu().numpy(), o.cpu().numpy()
    for k in range(4):
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 16, device=DEV).sum()
        torch.cuda.synchronize()
        f.fill_(float("nan"))
        o.fill_(float("nan"))
        b.forces(x, q, f=f, out7=o)
        torch.cuda.synchronize()
        assert _forces_close(f.double().cpu().numpy(), f0, 2e-6), k
        assert _close(o.cpu().numpy(), o0, 2e-6), k
        del junk
    # new positions in the same buffers: the replay sees them
    rng = np.random.default_rng(3)
    pos2 = [p + rng.normal(0, 0.01, p.shape) for p in pos]
    x.copy_(_cat(pos2, torch.float32))
    b.forces(x, q, f=f, out7=o)
    f2, o2 = f.double().cpu().numpy(), o.cpu().numpy()
    assert b.check() == esp.ESP_OK
    for r in (0, len(qs) - 1):
        fs, os_, _ = _single(cells, pos2, qs, tols, r, torch.float32)
        sl = slice(b.offsets[r], b.offsets[r + 1])
        assert _forces_close(f2[sl], fs, 2e-6)
        assert _close(o2[r], os_, 2e-6)
    b.close()


def test_batch_set_box(system):
    cells, pos, qs, tols = system
    ns = [len(q) for q in qs]
    b = esp.Batch(cells, ns, tols, graph=True, window_tol=1e-9)
    x, q = _cat(pos, torch.float32), _cat(qs, torch.float32)
    f, o = b.forces(x, q)
    b.forces(x, q, f=f, out7=o)                 # replay of the recorded graph
    r = 2
    h_new = cells[r] * 1.02
    b.set_box(r, h_new)
    b.forces(x, q, f=f, out7=o)                 # same graph, new cell of replica r
    f, o = f.double().cpu().numpy(), o.cpu().numpy()
    cells2 = list(cells)
    cells2[r] = h_new
    fs, os_, _ = _single(cells2, pos, qs, tols, r, torch.float32, prm=b.params[r], window_tol=1e-9)
    sl = slice(b.offsets[r], b.offsets[r + 1])
    assert _forces_close(f[sl], fs, 2e-6)
    assert _close(o[r], os_, 2e-6)
    # the other replicas are unchanged
    fs0, os0, _ = _single(cells, pos, qs, tols, 0, torch.float32, prm=b.params[0], window_tol=1e-9)
    assert _forces_close(f[slice(b.offsets[0], b.offsets[1])], fs0, 2e-6)
    assert _close(o[0], os0, 2e-6)
    b.close()
