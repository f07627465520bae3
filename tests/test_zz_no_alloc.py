"""The allocation-free entry point (esp_forces_noalloc: a plan carved out of
the library's static device scratch array) against esp_forces on an ordinary
plan with the same arguments, through the C ABI: two calls in a row, the
second smaller, each compared quantity by quantity."""

import numpy as np
import pytest

import gpu_util as gu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_00161_amd import esp, synth  # noqa: E402

DEV = "cuda:0"


def _triclinic_water(n_mol, L, seed):
    h = synth.cubic(L)
    h[0, 1], h[0, 2], h[1, 2] = 0.2 * L, -0.1 * L, 0.15 * L
    return synth.water(n_mol, h, config=1, seed=seed)


def _reference(h, r, q, tol, opts):
    """esp_forces on an esp_plan plan (the existing entry point)."""
    x = torch.from_numpy(np.ascontiguousarray(r, np.float32)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(DEV)
    plan = esp.Plan(h, len(q), tol, **opts)
    f, o = plan.forces(x, c)
    torch.cuda.synchronize()
    plan.check()
    out = f.cpu().numpy().astype(np.float64), o.cpu().numpy()
    plan.close()
    return out


CASES = [
    # (label, molecules, edge nm, tol, options): the first call is the larger
    ("triclinic_water_9000_flex_1e-5", 3000, 4.5, 1e-5, dict(coupling="flex")),
    ("triclinic_water_1500_1e-4", 500, 2.6, 1e-4, dict()),
]


def test_noalloc_matches_esp_forces_on_two_calls_in_a_row():
    results = []
    for k, (label, nmol, L, tol, opts) in enumerate(CASES):
        h, r, q = _triclinic_water(nmol, L, seed=k)
        print(f"noalloc case {label}: n={len(q)} tol={tol}", flush=True)
        x = torch.from_numpy(np.ascontiguousarray(r, np.float32)).to(DEV)
        c = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(DEV)
        # outputs hold garbage from before: the call overwrites every element
        f = torch.full((len(q), 3), float("nan"), dtype=torch.float32, device=DEV)
        o = torch.full((7,), float("nan"), dtype=torch.float64, device=DEV)
        esp.forces_noalloc(h, x, c, tol, f=f, out7=o, **opts)
        torch.cuda.synchronize()
        results.append((label, h, r, q, tol, opts, f.cpu().numpy().astype(np.float64), o.cpu().numpy()))
    # the references afterwards, so the second no-alloc call above ran right
    # behind the first, in the scratch the first one left
    for label, h, r, q, tol, opts, f, o in results:
        fr, orf = _reference(h, r, q, tol, opts)
        assert np.all(np.isfinite(f)) and np.all(np.isfinite(o)), label
        gu.parity(f"noalloc_{label}", o, orf[0], orf[1:], f, fr, "fp32")
        print(f"noalloc {label}: bit-identical out7 {np.array_equal(o, orf)} forces {np.array_equal(f, fr)}",
              flush=True)


def test_noalloc_same_system_twice_is_repeatable():
    """A call after a larger one on the same scratch gives the result of the
    first call of that size (nothing left over from the previous user), to the
    parity bar: the spreading's write-back adds tile boxes to the grid with
    float atomics, so the order of those additions, and the last bits of the
    grid, can change from run to run."""
    h, r, q = _triclinic_water(500, 2.6, seed=7)
    x = torch.from_numpy(np.ascontiguousarray(r, np.float32)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(DEV)
    f1, o1 = esp.forces_noalloc(h, x, c, 1e-4)
    torch.cuda.synchronize()
    f1, o1 = f1.cpu().numpy(), o1.cpu().numpy()
    h2, r2, q2 = _triclinic_water(2000, 4.0, seed=8)
    x2 = torch.from_numpy(np.ascontiguousarray(r2, np.float32)).to(DEV)
    c2 = torch.from_numpy(np.ascontiguousarray(q2, np.float32)).to(DEV)
    esp.forces_noalloc(h2, x2, c2, 1e-5)
    f3, o3 = esp.forces_noalloc(h, x, c, 1e-4)
    torch.cuda.synchronize()
    gu.parity("noalloc_repeat", o3.cpu().numpy(), o1[0], o1[1:], f3.cpu().numpy(), f1, "fp32")


def test_noalloc_refuses_a_plan_beyond_the_scratch_size():
    """3 x 10^6 particles need ~130 MB of buffers: ESP_ENOMEM, and the outputs
    are left as they were."""
    n = 3_000_000
    h = synth.cubic(30.0)
    x = torch.rand((n, 3), dtype=torch.float32, device=DEV) * 30.0
    c = torch.zeros(n, dtype=torch.float32, device=DEV)
    f = torch.full((n, 3), 7.0, dtype=torch.float32, device=DEV)
    o = torch.full((7,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(esp.EspError) as ei:
        esp.forces_noalloc(h, x, c, 1e-5, f=f, out7=o)
    assert ei.value.status == esp.ESP_ENOMEM
    torch.cuda.synchronize()
    assert bool(torch.all(f == 7.0)) and bool(torch.all(o == 7.0))


def test_noalloc_refuses_learned_parameters_and_fp64():
    h, r, q = _triclinic_water(100, 2.0, seed=3)
    x = torch.from_numpy(np.ascontiguousarray(r, np.float32)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(DEV)
    for opts in (dict(params="learned"), dict(precision="fp64"), dict(local_virial=True)):
        with pytest.raises(esp.EspError) as ei:
            esp.forces_noalloc(h, x, c, 1e-4, **opts)
        assert ei.value.status == esp.ESP_EINVAL


def test_noalloc_allocates_no_device_memory():
    """Free device memory is unchanged by calls after the first (which loads
    the code objects holding the scratch array)."""
    h, r, q = _triclinic_water(3000, 4.5, seed=5)
    x = torch.from_numpy(np.ascontiguousarray(r, np.float32)).to(DEV)
    c = torch.from_numpy(np.ascontiguousarray(q, np.float32)).to(DEV)
    f = torch.empty((len(q), 3), dtype=torch.float32, device=DEV)
    o = torch.empty(7, dtype=torch.float64, device=DEV)
    esp.forces_noalloc(h, x, c, 1e-5, f=f, out7=o)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for tol in (1e-5, 1e-4, 1e-6):
        esp.forces_noalloc(h, x, c, tol, f=f, out7=o)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"noalloc free device memory before {free0} after {free1}", flush=True)
    assert free0 - free1 < (1 << 20)
