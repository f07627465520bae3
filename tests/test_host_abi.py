"""CPU tests of the C ABI library: symbols, host-side parameter rules, PSWF
numerics and argument validation.  No GPU is used (no compute call is made)."""
import os
import re

import numpy as np
import pytest

from oracle.pswf import PSWF, c_from_tol
from paper_2601_00161_amd import esp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "esp.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(esp_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = esp.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    bound = {s[0] for s in esp.SIGNATURES}
    assert set(names) <= bound, set(names) - bound
    assert b"gfx950" in lib.esp_version()


def rule_M(h, c, rc, sigma=1.07):
    def smooth(m):
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        return m == 1
    out = []
    for d in range(3):
        m = int(np.ceil(sigma * np.linalg.norm(h[:, d]) * c / (np.pi * rc) - 1e-9))
        while not smooth(m):
            m += 1
        out.append(m)
    return out


@pytest.mark.parametrize("tol,coupling", [(1e-3, "iso"), (1e-4, "iso"), (1e-5, "semi"), (1e-5, "flex"),
                                          (1e-7, "aniso")])
def test_analytic_parameter_rule(tol, coupling):
    """c from psi(1)/psi(0) = Delta (the oracle's root), P = ceil(-log10 Delta) + 1,
    M from the grid rule, Delta = tol/5 when off-diagonal components are needed."""
    h = np.array([[9.0, 1.2, 0.8], [0.0, 9.0, 0.5], [0.0, 0.0, 9.0]])
    p = esp.resolve_params(h, 19200, tol, coupling=coupling)
    delta = tol / 5 if coupling == "flex" else tol
    assert p["delta"] == pytest.approx(delta, rel=1e-12)
    assert p["c_split"] == pytest.approx(c_from_tol(delta), rel=1e-9)
    assert p["c_spread"] == p["c_split"]
    assert p["P"] == int(np.ceil(-np.log10(delta) - 1e-9)) + 1
    assert p["M"] == rule_M(h, p["c_split"], 0.9)
    assert p["volume"] == pytest.approx(np.linalg.det(h))
    ps = PSWF(p["c_split"])
    assert p["lambda0_split"] == pytest.approx(ps.lam0, rel=1e-10)
    assert p["C0_split"] == pytest.approx(ps.C0, rel=1e-10)


def test_explicit_parameters_pass_through():
    p = esp.resolve_params(np.diag([3.0, 3.0, 3.0]), 100, 1e-4, c_split=11.0, c_spread=12.0, P=7, M=(16, 18, 20))
    assert p["params_source"] == 1
    assert (p["c_split"], p["c_spread"], p["P"], p["M"]) == (11.0, 12.0, 7, [16, 18, 20])


@pytest.mark.parametrize("c", [2.0, 11.68, 14.08, 25.0])
def test_library_pswf_matches_oracle(c):
    """Two independent implementations (C++ Sturm/inverse iteration vs the oracle's
    SciPy eigensolver) of the same function, both pinned to the eigen-equation."""
    x = np.array([-1.3, -0.7, 0.0, 0.2, 0.55, 0.9, 1.0, 1.25])
    psi, dpsi, ipsi, (psi0, C0, lam0) = esp.pswf_eval(c, x)
    o = PSWF(c)
    assert np.max(np.abs(psi - o.psi_ext(x))) < 1e-12
    assert np.max(np.abs(dpsi - o.dpsi_ext(x))) < 1e-10 * max(1.0, c)
    inside = np.abs(x) <= 1
    assert np.max(np.abs(ipsi[inside] - o.int_psi(x[inside]))) < 1e-13
    assert np.all(np.isnan(ipsi[~inside]))
    assert abs(psi0 - o.psi0) < 1e-13 and abs(C0 - o.C0) < 1e-13 and abs(lam0 - o.lam0) < 1e-12


def test_c_from_delta_matches_oracle():
    for d in (1e-3, 1e-5, 2e-6, 1e-9):
        assert esp.c_from_delta(d) == pytest.approx(c_from_tol(d), rel=1e-7)


@pytest.mark.parametrize("h,n,tol,kw,status", [
    (np.diag([3.0, 3.0, -3.0]), 10, 1e-4, {}, esp.ESP_EBOX),
    (np.diag([3.0, np.nan, 3.0]), 10, 1e-4, {}, esp.ESP_EBOX),
    (np.array([[3.0, 3.0, 0.0], [0.0, 0.0, 3.0], [0.0, 0.0, 0.0]]), 10, 1e-4, {}, esp.ESP_EBOX),
    (np.diag([1.5, 3.0, 3.0]), 10, 1e-4, {}, esp.ESP_ECUTOFF),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-4, {"rc": 1.6}, esp.ESP_ECUTOFF),
    (np.diag([3.0, 3.0, 3.0]), 0, 1e-4, {}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 0.5, {}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-13, {}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-4, {"c_split": 11.0, "P": 5, "M": (14, 15, 15)}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-4, {"c_split": 11.0, "P": 13, "M": 16}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-4, {"c_split": 11.0, "P": 6, "M": 5}, esp.ESP_EINVAL),
    (np.diag([3.0, 3.0, 3.0]), 10, 1e-4, {"precision": 7}, esp.ESP_EINVAL),
])
def test_argument_validation(h, n, tol, kw, status):
    with pytest.raises(esp.EspError) as ei:
        esp.resolve_params(h, n, tol, **kw)
    assert ei.value.status == status


def test_tiny_cell_rule_respects_support():
    """Grids never get fewer points than the window support."""
    p = esp.resolve_params(np.diag([1.9, 1.9, 1.9]), 12, 1e-7)
    assert min(p["M"]) >= p["P"]


def test_learned_without_proposer_falls_back_to_analytic():
    """No registered network: ESP_LEARNED resolves to the analytic rule with a
    warning status (called through the C ABI directly; the Python binding
    would register the shipped weights, which needs a GPU)."""
    import ctypes
    lib = esp.lib()
    assert lib.esp_proposer_set(None) == esp.ESP_OK
    h = np.diag([6.7, 6.7, 6.7])
    hp = np.ascontiguousarray(h)
    o = esp.make_opts(params="learned")
    out = esp.Params()
    st = lib.esp_resolve_params(hp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 30000, 1e-5,
                                ctypes.byref(o), ctypes.byref(out))
    assert st == esp.ESP_WARN_FALLBACK
    ana = esp.resolve_params(h, 30000, 1e-5)
    got = out.as_dict()
    assert got["params_source"] == esp.PARAMS["analytic"]
    for k in ("delta", "c_split", "P", "M"):
        assert got[k] == ana[k]
    assert list(got["predicted_log10_err"]) == [0.0] * 4


def test_proposer_registration_rejects_missing_network():
    p = esp.Proposer()
    for i in range(esp.PROPOSER_FEATURES):
        p.in_std[i] = 1.0
    for i in range(4):
        p.out_std[i] = 1.0
    assert esp.lib().esp_proposer_set(p) == esp.ESP_EINVAL


def test_autotune_cache_key():
    from paper_2601_00161_amd import autotune
    k = autotune._key({"n": 31234, "precision": 0, "M": [36, 36, 40], "P": 6, "window_degree": 9})
    assert k == "fp32:M36x36x40:P6:W12:N31000"
    assert autotune._key({"n": 987, "precision": 1, "M": [15, 15, 15], "P": 5, "window_degree": 14}) == \
        "fp64:M15x15x15:P5:W16:N990"


def test_gather_option_is_validated():
    with pytest.raises(esp.EspError):
        esp.resolve_params(np.diag([3.0, 3.0, 3.0]), 100, 1e-4, gather=7)


def test_force_option_is_validated():
    with pytest.raises(esp.EspError):
        esp.resolve_params(np.diag([3.0, 3.0, 3.0]), 100, 1e-4, force=5)
    assert esp.resolve_params(np.diag([3.0, 3.0, 3.0]), 100, 1e-4, force="ik")["P"] >= 2


def test_fp32_below_its_floor_warns():
    """An FP32 plan asked for tol < 1e-6 is planned (the rule's parameters) but
    flagged ESP_WARN_PRECISION; FP64 plans and FP32 at 1e-6 are not."""
    import ctypes
    h = np.diag([3.0, 3.0, 3.0])
    hp = np.ascontiguousarray(h).ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for prec, tol, want in (("fp32", 1e-7, esp.ESP_WARN_PRECISION), ("fp32", 1e-6, esp.ESP_OK),
                            ("fp64", 1e-7, esp.ESP_OK), ("fp32", 1e-5, esp.ESP_OK)):
        o = esp.make_opts(precision=prec)
        out = esp.Params()
        st = esp.lib().esp_resolve_params(hp, 3000, tol, ctypes.byref(o), ctypes.byref(out))
        assert st == want, (prec, tol, st)
        assert out.P == int(np.ceil(-np.log10(tol) - 1e-9)) + 1
