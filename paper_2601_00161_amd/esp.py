"""Thin Python binding of the C ABI in ``include/esp.h``.

Argument marshalling only: every step of the path runs in the HIP library
``libesp_mi355x.so``.  PyTorch supplies device memory and the current stream;
no torch type crosses the C boundary (pointers and sizes only).  If the
library is missing the calls raise; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesp_mi355x.so")

ESP_OK, ESP_WARN_REPLAN, ESP_WARN_FALLBACK, ESP_WARN_PRECISION = 0, 1, 2, 3
ESP_EINVAL, ESP_EBOX, ESP_ECUTOFF, ESP_ENOMEM, ESP_EDEVICE, ESP_ENONFINITE = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "ESP_OK", 1: "ESP_WARN_REPLAN", 2: "ESP_WARN_FALLBACK", 3: "ESP_WARN_PRECISION", -1: "ESP_EINVAL",
                -2: "ESP_EBOX", -3: "ESP_ECUTOFF", -4: "ESP_ENOMEM", -5: "ESP_EDEVICE",
                -6: "ESP_ENONFINITE"}
PRECISION = {"fp32": 0, "fp64": 1}
PARAMS = {"analytic": 0, "explicit": 1, "learned": 2}
COUPLING = {"iso": 0, "semi": 1, "aniso": 2, "flex": 3}
GATHER = {"auto": 0, "particle": 1, "tile": 2, "lane": 3}
FORCE = {"ad": 0, "ik": 1}
SPREAD_ACCUM = {"auto": 0, "fixed": 1, "fp64": 2}


class EspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("params", ctypes.c_int), ("coupling", ctypes.c_int),
                ("rc", ctypes.c_double), ("c_split", ctypes.c_double), ("c_spread", ctypes.c_double),
                ("P", ctypes.c_int), ("M", ctypes.c_int * 3), ("grid_sigma", ctypes.c_double),
                ("coulomb_k", ctypes.c_double), ("tile", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("window_tol", ctypes.c_double), ("gather", ctypes.c_int), ("force", ctypes.c_int),
                ("local_virial", ctypes.c_int), ("fft_split", ctypes.c_int), ("spread_accum", ctypes.c_int),
                ("deterministic", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("n", ctypes.c_int64), ("tol", ctypes.c_double),
                ("delta", ctypes.c_double), ("rc", ctypes.c_double), ("c_split", ctypes.c_double),
                ("c_spread", ctypes.c_double), ("P", ctypes.c_int), ("M", ctypes.c_int * 3),
                ("tile", ctypes.c_int * 3), ("ntiles", ctypes.c_int), ("window_degree", ctypes.c_int),
                ("kernel_degree", ctypes.c_int), ("lambda0_split", ctypes.c_double),
                ("C0_split", ctypes.c_double), ("psi0_split", ctypes.c_double),
                ("volume", ctypes.c_double), ("params_source", ctypes.c_int),
                ("predicted_log10_err", ctypes.c_double * 4), ("predicted_cost", ctypes.c_double),
                ("gather_tiled", ctypes.c_int), ("counter_copies", ctypes.c_int), ("force", ctypes.c_int),
                ("local_virial", ctypes.c_int), ("real_cells", ctypes.c_int * 3),
                ("real_segments", ctypes.c_int), ("fft_split", ctypes.c_int), ("spread_fixed", ctypes.c_int),
                ("hinv", ctypes.c_double * 9), ("gather_lane", ctypes.c_int),
                ("grid_fixed", ctypes.c_int)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, ctypes.Array) else v
        return out


PROPOSER_FEATURES = 4


class Proposer(ctypes.Structure):
    _fields_ = [("mlp", ctypes.c_void_p), ("in_mean", ctypes.c_double * PROPOSER_FEATURES),
                ("in_std", ctypes.c_double * PROPOSER_FEATURES), ("out_mean", ctypes.c_double * 4),
                ("out_std", ctypes.c_double * 4), ("margin", ctypes.c_double * 4), ("cost", ctypes.c_double * 5)]


# (name, restype, argtypes) of every exported symbol declared in include/esp.h
_P = ctypes.c_void_p
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("esp_opts_default", None, [ctypes.POINTER(Opts)]),
    ("esp_plan", ctypes.c_int, [_DP, ctypes.c_int64, _D, ctypes.POINTER(Opts), ctypes.POINTER(_P)]),
    ("esp_set_box", ctypes.c_int, [_P, _DP]),
    ("esp_energy_virial", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_energy_virial_f64", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_forces", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_forces_f64", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_forces_noalloc", ctypes.c_int, [_DP, ctypes.c_int64, _D, ctypes.POINTER(Opts), _P, _P, _P, _P]),
    ("esp_check", ctypes.c_int, [_P]),
    ("esp_local_virial", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_local_virial_f64", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_real_space", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P]),
    ("esp_real_space_f64", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _P]),
    ("esp_coulomb", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_coulomb_f64", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_get_params", ctypes.c_int, [_P, ctypes.POINTER(Params)]),
    ("esp_last_error", ctypes.c_char_p, [_P]),
    ("esp_destroy", None, [_P]),
    ("esp_stage_sort", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_stage_spread", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_stage_fft", ctypes.c_int, [_P, _P, _P]),
    ("esp_stage_potential", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_set_stream", ctypes.c_int, [_P, _P]),
    ("esp_resolve_params", ctypes.c_int, [_DP, ctypes.c_int64, _D, ctypes.POINTER(Opts), ctypes.POINTER(Params)]),
    ("esp_pswf_eval", ctypes.c_int, [_D, ctypes.c_int64, _DP, _DP, _DP, _DP, _DP]),
    ("esp_c_from_delta", ctypes.c_double, [_D]),
    ("esp_profile_enable", ctypes.c_int, [_P, ctypes.c_uint, ctypes.c_int, ctypes.c_int]),
    ("esp_profile_read", ctypes.c_int, [_P, _DP, ctypes.POINTER(ctypes.c_int64)]),
    ("esp_stage_name", ctypes.c_char_p, [ctypes.c_int]),
    ("esp_mlp_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_uint64,
                                      ctypes.POINTER(_P)]),
    ("esp_mlp_num_params", ctypes.c_int64, [_P]),
    ("esp_mlp_set_params", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("esp_mlp_get_params", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("esp_mlp_set_stream", ctypes.c_int, [_P, _P]),
    ("esp_mlp_forward", ctypes.c_int, [_P, _P, ctypes.c_int64, _P]),
    ("esp_mlp_gradient", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, _P, _P]),
    ("esp_mlp_train_step", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_float, _P]),
    ("esp_mlp_destroy", None, [_P]),
    ("esp_proposer_set", ctypes.c_int, [ctypes.POINTER(Proposer)]),
    ("esp_batch_plan", ctypes.c_int, [ctypes.c_int, _DP, ctypes.POINTER(ctypes.c_int64), _DP,
                                      ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_P)]),
    ("esp_batch_energy_virial", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_batch_forces", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_batch_energy_virial_f64", ctypes.c_int, [_P, _P, _P, _P]),
    ("esp_batch_forces_f64", ctypes.c_int, [_P, _P, _P, _P, _P]),
    ("esp_batch_set_box", ctypes.c_int, [_P, ctypes.c_int, _DP]),
    ("esp_batch_set_stream", ctypes.c_int, [_P, _P]),
    ("esp_batch_set_graph", ctypes.c_int, [_P, ctypes.c_int]),
    ("esp_batch_check", ctypes.c_int, [_P]),
    ("esp_batch_get_params", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(Params)]),
    ("esp_batch_num_launches", ctypes.c_int, [_P, ctypes.c_int]),
    ("esp_batch_last_error", ctypes.c_char_p, [_P]),
    ("esp_batch_destroy", None, [_P]),
    ("esp_version", ctypes.c_char_p, []),
]
NUM_STAGES = 8

_lib_handle = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2601_00161_amd.build` (there is no fallback)")
        h = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib_handle = h
    return _lib_handle


def _cell(h):
    a = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(3, 3))
    return a, a.ctypes.data_as(_DP)


def make_opts(precision="fp32", params="analytic", coupling="iso", rc=0.9, c_split=None,
              c_spread=None, P=None, M=None, grid_sigma=1.07, coulomb_k=1.0, tile=0, stream=None,
              window_tol=0.0, gather="auto", force="ad", local_virial=False, fft_split=False,
              spread_accum="auto", deterministic=False):
    o = Opts()
    lib().esp_opts_default(ctypes.byref(o))
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    explicit = any(v is not None for v in (c_split, c_spread, P, M))
    if explicit and params == "analytic":
        params = "explicit"
    o.params = PARAMS[params] if isinstance(params, str) else int(params)
    o.coupling = COUPLING[coupling] if isinstance(coupling, str) else int(coupling)
    o.rc = rc
    if c_split is not None:
        o.c_split = c_split
        o.c_spread = c_split if c_spread is None else c_spread
    elif c_spread is not None:
        o.c_spread = c_spread
    if P is not None:
        o.P = int(P)
    if M is not None:
        M = [int(M)] * 3 if np.isscalar(M) else [int(m) for m in M]
        for d in range(3):
            o.M[d] = M[d]
    o.grid_sigma = grid_sigma
    o.coulomb_k = coulomb_k
    o.tile = int(tile)
    o.stream = stream
    o.window_tol = float(window_tol)
    o.gather = GATHER[gather] if isinstance(gather, str) else int(gather)
    o.force = FORCE[force] if isinstance(force, str) else int(force)
    o.local_virial = 1 if local_virial else 0
    o.fft_split = 1 if fft_split else 0
    o.spread_accum = SPREAD_ACCUM[spread_accum] if isinstance(spread_accum, str) else int(spread_accum)
    o.deterministic = 1 if deterministic else 0
    return o


def resolve_params(h, n, tol, **opts):
    """Parameters esp_plan would choose (host only, no device needed)."""
    o = make_opts(**opts)
    if o.params == PARAMS["learned"]:
        from . import learned
        learned.ensure_default()
    _, hp = _cell(h)
    out = Params()
    st = lib().esp_resolve_params(hp, int(n), float(tol), ctypes.byref(o), ctypes.byref(out))
    if st < 0:
        raise EspError(st, "esp_resolve_params rejected the arguments")
    return out.as_dict()


def pswf_eval(c, x):
    """psi_0^c, its derivative and integral at x; returns (psi, dpsi, ipsi, (psi0, C0, lambda0))."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    psi, dpsi, ipsi = (np.empty_like(x) for _ in range(3))
    k = np.empty(3)
    st = lib().esp_pswf_eval(float(c), x.size, x.ctypes.data_as(_DP), psi.ctypes.data_as(_DP),
                             dpsi.ctypes.data_as(_DP), ipsi.ctypes.data_as(_DP), k.ctypes.data_as(_DP))
    if st != ESP_OK:
        raise EspError(st, "esp_pswf_eval")
    return psi, dpsi, ipsi, tuple(k)


def c_from_delta(delta):
    return float(lib().esp_c_from_delta(float(delta)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


NOALLOC_SCRATCH_BYTES = 96 << 20


def forces_noalloc(h, xyz, q, tol, f=None, out7=None, **opts):
    """esp_forces_noalloc: plan + forces in the library's static device scratch
    (no device allocation by the library); FP32 tensors on the GPU, enqueued on
    torch's current stream.  Returns (f, out7); pass f / out7 to reuse buffers."""
    import torch
    if not (xyz.is_cuda and q.is_cuda) or xyz.dtype != torch.float32 or q.dtype != torch.float32:
        raise ValueError("xyz and q must be float32 device tensors")
    if not (xyz.is_contiguous() and q.is_contiguous()) or xyz.numel() != 3 * q.numel():
        raise ValueError("expected contiguous xyz of 3 n and q of n elements")
    n = q.numel()
    if f is None:
        f = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    if out7 is None:
        out7 = torch.empty(7, dtype=torch.float64, device=xyz.device)
    o = make_opts(**opts, stream=ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _, hp = _cell(h)
    st = lib().esp_forces_noalloc(hp, n, float(tol), ctypes.byref(o), _ptr(xyz), _ptr(q), _ptr(f), _ptr(out7))
    if st < 0:
        raise EspError(st, "esp_forces_noalloc failed (see stderr)")
    return f, out7


class Plan:
    """An ESP plan for n particles in cell h at tolerance tol (device memory owned here).

    The call methods take torch tensors on the GPU (contiguous, float32 for an
    fp32 plan, float64 for fp64) and enqueue on torch's current stream.
    """

    def __init__(self, h, n, tol, **opts):
        import torch  # device memory and streams only
        self._torch = torch
        self._lib = lib()
        o = make_opts(**opts)
        if o.params == PARAMS["learned"]:
            from . import learned
            learned.ensure_default()
        _, hp = _cell(h)
        handle = ctypes.c_void_p()
        st = self._lib.esp_plan(hp, int(n), float(tol), ctypes.byref(o), ctypes.byref(handle))
        if st < 0:
            raise EspError(st, "esp_plan failed (see stderr)")
        self.status = st
        self._h = handle
        self.n = int(n)
        prm = Params()
        self._lib.esp_get_params(self._h, ctypes.byref(prm))
        self.params = prm.as_dict()
        self.dtype = torch.float32 if self.params["precision"] == 0 else torch.float64

    # -- helpers -------------------------------------------------------------
    def _err(self, st, what):
        msg = self._lib.esp_last_error(self._h)
        raise EspError(st, f"{what}: {msg.decode() if msg else ''}")

    def _stream(self):
        s = self._torch.cuda.current_stream().cuda_stream
        self._lib.esp_set_stream(self._h, ctypes.c_void_p(s))

    def _check_in(self, xyz, q):
        t = self._torch
        if not (xyz.is_cuda and q.is_cuda):
            raise ValueError("xyz and q must be device tensors")
        if xyz.dtype != self.dtype or q.dtype != self.dtype:
            raise ValueError(f"inputs must be {self.dtype}")
        if xyz.numel() != 3 * self.n or q.numel() != self.n:
            raise ValueError(f"expected xyz of {3 * self.n} and q of {self.n} elements")
        if not (xyz.is_contiguous() and q.is_contiguous()):
            raise ValueError("inputs must be contiguous")
        return t

    # -- the path ------------------------------------------------------------
    def set_box(self, h):
        _, hp = _cell(h)
        st = self._lib.esp_set_box(self._h, hp)
        if st < 0:
            self._err(st, "esp_set_box")
        prm = Params()
        self._lib.esp_get_params(self._h, ctypes.byref(prm))
        self.params = prm.as_dict()
        return st

    def energy_virial(self, xyz, q, out7=None):
        t = self._check_in(xyz, q)
        if out7 is None:
            out7 = t.empty(7, dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_energy_virial if self.dtype == t.float32 else self._lib.esp_energy_virial_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(out7))
        if st < 0:
            self._err(st, "esp_energy_virial")
        return out7

    def forces(self, xyz, q, f=None, out7=None, want_energy=True):
        t = self._check_in(xyz, q)
        if f is None:
            f = t.empty((self.n, 3), dtype=self.dtype, device=xyz.device)
        if out7 is None and want_energy:
            out7 = t.empty(7, dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_forces if self.dtype == t.float32 else self._lib.esp_forces_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(f), _ptr(out7) if out7 is not None else None)
        if st < 0:
            self._err(st, "esp_forces")
        return f, out7

    def local_virial(self, xyz, q, w6=None, out7=None):
        """Per-particle Fourier virial, (n, 6) in xx, yy, zz, xy, xz, yz order."""
        t = self._check_in(xyz, q)
        if w6 is None:
            w6 = t.empty((self.n, 6), dtype=self.dtype, device=xyz.device)
        self._stream()
        fn = self._lib.esp_local_virial if self.dtype == t.float32 else self._lib.esp_local_virial_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(w6), _ptr(out7) if out7 is not None else None)
        if st < 0:
            self._err(st, "esp_local_virial")
        return w6, out7

    def real_space(self, xyz, q, f=None, out7=None, accumulate=False):
        """Near part over pairs within rc: forces (n, 3) (added to f when
        accumulate) and out7 = (U_N, W_N) in the Fourier part's layout."""
        t = self._check_in(xyz, q)
        if f is None:
            if accumulate:
                raise ValueError("accumulate needs an f to add to")
            f = t.empty((self.n, 3), dtype=self.dtype, device=xyz.device)
        if out7 is None:
            out7 = t.empty(7, dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_real_space if self.dtype == t.float32 else self._lib.esp_real_space_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(f), 1 if accumulate else 0, _ptr(out7))
        if st < 0:
            self._err(st, "esp_real_space")
        return f, out7

    def coulomb(self, xyz, q, f=None, out7=None):
        """Total Coulomb forces (n, 3) and out7 (near plus Fourier energy
        and virial); the near part runs on a second stream beside the
        Fourier part."""
        t = self._check_in(xyz, q)
        if f is None:
            f = t.empty((self.n, 3), dtype=self.dtype, device=xyz.device)
        if out7 is None:
            out7 = t.empty(7, dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_coulomb if self.dtype == t.float32 else self._lib.esp_coulomb_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(f), _ptr(out7))
        if st < 0:
            self._err(st, "esp_coulomb")
        return f, out7

    def check(self):
        st = self._lib.esp_check(self._h)
        if st < 0:
            self._err(st, "esp_check")
        return st

    # -- stage hooks -----------------------------------------------------------
    def stage_sort(self, xyz, q):
        t = self._check_in(xyz, q)
        perm = t.empty(self.n, dtype=t.int32, device=xyz.device)
        off = t.empty(self.params["ntiles"] + 1, dtype=t.int32, device=xyz.device)
        self._stream()
        st = self._lib.esp_stage_sort(self._h, _ptr(xyz), _ptr(q), _ptr(perm), _ptr(off))
        if st < 0:
            self._err(st, "esp_stage_sort")
        return perm, off

    def grid_shape(self):
        M = self.params["M"]
        return (M[2], M[1], M[0])          # g1 fastest

    def stage_spread(self, xyz, q):
        t = self._check_in(xyz, q)
        g = t.empty(self.grid_shape(), dtype=self.dtype, device=xyz.device)
        self._stream()
        st = self._lib.esp_stage_spread(self._h, _ptr(xyz), _ptr(q), _ptr(g))
        if st < 0:
            self._err(st, "esp_stage_spread")
        return g

    def stage_fft(self, grid):
        t = self._torch
        M = self.params["M"]
        if grid.dtype != self.dtype or tuple(grid.shape) != self.grid_shape() or not grid.is_contiguous():
            raise ValueError("grid must be a contiguous (M3, M2, M1) tensor of the plan's dtype")
        cdt = t.complex64 if self.dtype == t.float32 else t.complex128
        spec = t.empty((M[2], M[1], M[0] // 2 + 1), dtype=cdt, device=grid.device)
        self._stream()
        st = self._lib.esp_stage_fft(self._h, _ptr(grid), _ptr(spec))
        if st < 0:
            self._err(st, "esp_stage_fft")
        return spec

    def stage_potential(self, xyz, q):
        t = self._check_in(xyz, q)
        phi = t.empty(self.grid_shape(), dtype=self.dtype, device=xyz.device)
        self._stream()
        st = self._lib.esp_stage_potential(self._h, _ptr(xyz), _ptr(q), _ptr(phi))
        if st < 0:
            self._err(st, "esp_stage_potential")
        return phi

    # -- per-stage timing ------------------------------------------------------
    def profile(self, stages, max_launches, stride=1):
        """Record HIP events around every stride-th launch of the named stages."""
        names = [self._lib.esp_stage_name(i).decode() for i in range(NUM_STAGES)]
        mask = 0
        for s in stages:
            mask |= 1 << names.index(s)
        st = self._lib.esp_profile_enable(self._h, mask, int(max_launches), int(stride))
        if st < 0:
            self._err(st, "esp_profile_enable")

    def profile_read(self):
        """{stage: (total_ms, launches)} since profiling was enabled."""
        ms = (ctypes.c_double * NUM_STAGES)()
        cnt = (ctypes.c_int64 * NUM_STAGES)()
        st = self._lib.esp_profile_read(self._h, ms, cnt)
        if st < 0:
            self._err(st, "esp_profile_read")
        return {self._lib.esp_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NUM_STAGES) if cnt[i]}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.esp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent replicas evaluated together (one launch per stage).

    ``cells``: sequence of 3x3 cells; ``ns``: particle counts; ``tols``:
    tolerances.  Inputs are the replicas' arrays concatenated in order (torch
    CUDA tensors); ``out7`` is (nrep, 7).
    """

    def __init__(self, cells, ns, tols, tiles=None, graph=False, **opts):
        import torch
        self._torch = torch
        self._lib = lib()
        o = make_opts(**opts)
        if o.params == PARAMS["learned"]:
            from . import learned
            learned.ensure_default()
        self.nrep = len(ns)
        if not (len(cells) == len(tols) == self.nrep):
            raise ValueError("cells, ns and tols must have one entry per replica")
        h = np.ascontiguousarray(np.stack([np.asarray(c, np.float64).reshape(3, 3) for c in cells]))
        n = np.ascontiguousarray(np.asarray(ns, np.int64))
        tl = np.ascontiguousarray(np.asarray(tols, np.float64))
        tp = None
        if tiles is not None:
            ta = (ctypes.c_int * self.nrep)(*[int(t) for t in tiles])
            tp = ctypes.cast(ta, ctypes.POINTER(ctypes.c_int))
        handle = ctypes.c_void_p()
        st = self._lib.esp_batch_plan(self.nrep, h.ctypes.data_as(_DP), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      tl.ctypes.data_as(_DP), ctypes.byref(o), tp, ctypes.byref(handle))
        if st < 0:
            raise EspError(st, "esp_batch_plan failed (see stderr)")
        self.status = st
        self._h = handle
        self.ns = [int(v) for v in ns]
        self.offsets = np.concatenate([[0], np.cumsum(self.ns)]).astype(np.int64)
        self.params = []
        for r in range(self.nrep):
            prm = Params()
            self._lib.esp_batch_get_params(self._h, r, ctypes.byref(prm))
            self.params.append(prm.as_dict())
        self.dtype = torch.float32 if self.params[0]["precision"] == 0 else torch.float64
        if graph:
            self.set_graph(True)

    def _err(self, st, what):
        msg = self._lib.esp_batch_last_error(self._h)
        raise EspError(st, f"{what}: {msg.decode() if msg else ''}")

    def _stream(self):
        s = self._torch.cuda.current_stream().cuda_stream
        self._lib.esp_batch_set_stream(self._h, ctypes.c_void_p(s))

    def _check_in(self, xyz, q):
        t = self._torch
        N = int(self.offsets[-1])
        for a, shape in ((xyz, (N, 3)), (q, (N,))):
            if not a.is_cuda or a.dtype != self.dtype or tuple(a.shape) != shape or not a.is_contiguous():
                raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor of shape {shape}")
        return t

    def set_graph(self, enable):
        st = self._lib.esp_batch_set_graph(self._h, 1 if enable else 0)
        if st < 0:
            self._err(st, "esp_batch_set_graph")

    def num_launches(self, forces=True):
        return int(self._lib.esp_batch_num_launches(self._h, 1 if forces else 0))

    def energy_virial(self, xyz, q, out7=None):
        t = self._check_in(xyz, q)
        if out7 is None:
            out7 = t.empty((self.nrep, 7), dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_batch_energy_virial if self.dtype == t.float32 else self._lib.esp_batch_energy_virial_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(out7))
        if st < 0:
            self._err(st, "esp_batch_energy_virial")
        return out7

    def forces(self, xyz, q, f=None, out7=None, want_energy=True):
        t = self._check_in(xyz, q)
        if f is None:
            f = t.empty((int(self.offsets[-1]), 3), dtype=self.dtype, device=xyz.device)
        if out7 is None and want_energy:
            out7 = t.empty((self.nrep, 7), dtype=t.float64, device=xyz.device)
        self._stream()
        fn = self._lib.esp_batch_forces if self.dtype == t.float32 else self._lib.esp_batch_forces_f64
        st = fn(self._h, _ptr(xyz), _ptr(q), _ptr(f), _ptr(out7) if out7 is not None else None)
        if st < 0:
            self._err(st, "esp_batch_forces")
        return f, out7

    def set_box(self, r, h):
        _, hp = _cell(h)
        self._stream()
        st = self._lib.esp_batch_set_box(self._h, int(r), hp)
        if st < 0:
            self._err(st, "esp_batch_set_box")
        return st

    def check(self):
        st = self._lib.esp_batch_check(self._h)
        if st < 0:
            self._err(st, "esp_batch_check")
        return st

    def close(self):
        if getattr(self, "_h", None):
            self._lib.esp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
