"""Learned parameter proposer: binding of the library's MLP, its training on
the GPU, the cost-model calibration and the registration with the planner.

The network maps four features of a candidate parameter set and of the
system (log10 Delta, P, sigma and log10 of the charge density n/V) to the
predicted log10 relative errors of the total Coulomb energy, the diagonal and
off-diagonal pressure and the RMS force.  The cell shape enters through the
grid rule, which sizes M_d per cell vector; cell anisotropy and tilt as
features made predictions on held-out systems worse in grouped
cross-validation, so they are not used.  At plan time the library scores its
candidate grid with this network on the GPU and keeps the cheapest candidate,
under a fitted cost model, whose predictions meet the tolerance with a
per-output safety margin (a high quantile of the under-prediction in grouped
cross-validation over the training systems); if none does it takes the
candidate with the smallest predicted excess (the analytic rule's own choice
is one of the candidates) and warns.  The real-space cutoff stays fixed (rc
is an input), so
the proposer cannot trade reciprocal work for real-space work.

Training data are error labels measured against classical Ewald on small
synthetic systems (``tests/golden/proposer_data.json``); forward, backward
and Adam steps run in the library's own HIP kernels.  Commands::

    python -m paper_2601_00161_amd.learned train --data tests/golden/proposer_data.json --out W.json
    python -m paper_2601_00161_amd.learned cost --out W.json        # GPU timing sweep, adds cost

Weights ship as ``proposer_weights.json`` next to this file.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import time

import numpy as np

from . import esp

_HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(_HERE, "proposer_weights.json")
FEATURES = ("log10_delta", "P", "sigma", "log10_density")
OUTPUTS = ("energy", "pressure_diag", "pressure_offdiag", "force_rms")
LOG10_FLOOR = -10.0          # labels below this carry no information for the decision


class Mlp:
    """Owner of one esp_mlp_t (parameters live in device memory)."""

    def __init__(self, dims, seed=1):
        import torch
        self._torch = torch
        self._lib = esp.lib()
        self.dims = [int(d) for d in dims]
        arr = (ctypes.c_int * len(self.dims))(*self.dims)
        h = ctypes.c_void_p()
        st = self._lib.esp_mlp_create(len(self.dims) - 1, arr, ctypes.c_uint64(int(seed)), ctypes.byref(h))
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_create")
        self._h = h
        self.num_params = int(self._lib.esp_mlp_num_params(self._h))

    def _sync_stream(self):
        s = self._torch.cuda.current_stream().cuda_stream
        self._lib.esp_mlp_set_stream(self._h, ctypes.c_void_p(s))

    def get_params(self):
        out = np.empty(self.num_params, np.float32)
        self._torch.cuda.current_stream().synchronize()
        st = self._lib.esp_mlp_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p), self.num_params)
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_get_params")
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(np.asarray(w, np.float32))
        if w.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {w.size}")
        st = self._lib.esp_mlp_set_params(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size)
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_set_params")

    def _check(self, x, cols):
        t = self._torch
        if not (x.is_cuda and x.dtype == t.float32 and x.is_contiguous() and x.dim() == 2 and x.shape[1] == cols):
            raise ValueError(f"expected a contiguous float32 CUDA tensor of shape (B, {cols})")

    def forward(self, x):
        self._check(x, self.dims[0])
        y = self._torch.empty((x.shape[0], self.dims[-1]), device=x.device, dtype=self._torch.float32)
        self._sync_stream()
        st = self._lib.esp_mlp_forward(self._h, esp._ptr(x), x.shape[0], esp._ptr(y))
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_forward")
        return y

    def gradient(self, x, t, mask=None):
        """(gradient of the masked MSE over the flat parameters, loss) as device tensors."""
        self._check(x, self.dims[0])
        self._check(t, self.dims[-1])
        if mask is not None:
            self._check(mask, self.dims[-1])
        g = self._torch.empty(self.num_params, device=x.device, dtype=self._torch.float32)
        loss = self._torch.empty(1, device=x.device, dtype=self._torch.float32)
        self._sync_stream()
        st = self._lib.esp_mlp_gradient(self._h, esp._ptr(x), esp._ptr(t),
                                        None if mask is None else esp._ptr(mask), x.shape[0],
                                        esp._ptr(g), esp._ptr(loss))
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_gradient")
        return g, loss

    def train_step(self, x, t, lr, mask=None, loss=None):
        self._sync_stream()
        st = self._lib.esp_mlp_train_step(self._h, esp._ptr(x), esp._ptr(t),
                                          None if mask is None else esp._ptr(mask), x.shape[0],
                                          ctypes.c_float(lr), None if loss is None else esp._ptr(loss))
        if st != esp.ESP_OK:
            raise esp.EspError(st, "esp_mlp_train_step")

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            self._lib.esp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- features
def system_features(h, n):
    """(log10 n/V, anisotropy, tilt) of a cell h (columns are cell vectors)."""
    h = np.asarray(h, np.float64)
    V = abs(np.linalg.det(h))
    edges = np.linalg.norm(h, axis=0)
    tilt = max(abs(np.dot(h[:, a], h[:, b])) / (edges[a] * edges[b]) for a, b in ((0, 1), (0, 2), (1, 2)))
    return float(np.log10(n / V)), float(edges.max() / edges.min()), float(tilt)


def table(rows):
    """Feature matrix (R, 4) and clipped log10-error targets (R, 4) of data rows."""
    X = np.array([[np.log10(r["delta"]), r["P"], r["sigma"], r["log10_density"]] for r in rows], np.float64)
    Y = np.maximum(np.array([r["log10_err"] for r in rows], np.float64), LOG10_FLOOR)
    return X, Y


def _data_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# ---------------------------------------------------------------- training
def _fit(X, Y, hidden, steps, lr, seed):
    """Train one network on the GPU; returns (net, in/out normalisation, loss)."""
    import torch
    in_mean, in_std = X.mean(0), X.std(0)
    in_std[in_std == 0] = 1.0
    out_mean, out_std = Y.mean(0), Y.std(0)
    dev = torch.device("cuda:0")
    xt = torch.tensor((X - in_mean) / in_std, dtype=torch.float32, device=dev)
    yt = torch.tensor((Y - out_mean) / out_std, dtype=torch.float32, device=dev)
    net = Mlp([X.shape[1], *hidden, Y.shape[1]], seed=seed)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    for it in range(steps):
        # constant rate, then a geometric decay by 10x over the second half
        rate = lr if it < steps // 2 else lr * 0.1 ** ((it - steps // 2) / (steps // 2))
        net.train_step(xt, yt, rate, loss=loss)
    norm = (in_mean, in_std, out_mean, out_std)
    return net, norm, float(loss.item())


def _predict(net, norm, X):
    import torch
    in_mean, in_std, out_mean, out_std = norm
    xr = torch.tensor((X - in_mean) / in_std, dtype=torch.float32, device="cuda:0")
    return net.forward(xr).double().cpu().numpy() * out_std + out_mean


def train(data_path, hidden=(16, 16), steps=2000, lr=3e-3, seed=7, folds=5, quantile=0.995, holdout=()):
    """Train on the GPU.  The per-output margins are the `quantile` of the
    under-prediction (label - prediction) over rows near the decision region
    in grouped `folds`-fold cross-validation (whole systems held out); the
    final network is then trained on every system not in `holdout`."""
    with open(data_path) as f:
        data = json.load(f)
    rows = [r for r in data["rows"] if r["system"] not in holdout]
    systems = sorted({r["system"] for r in rows})
    order = np.random.default_rng(seed).permutation(len(systems))
    res = []
    for k in range(folds):
        test = {systems[i] for i in order[k::folds]}
        Xa, Ya = table([r for r in rows if r["system"] not in test])
        Xb, Yb = table([r for r in rows if r["system"] in test])
        net, norm, _ = _fit(Xa, Ya, hidden, steps, lr, seed)
        res.append((Yb, Yb - _predict(net, norm, Xb)))
        net.close()
        print(f"fold {k + 1}/{folds}: held out {sorted(test)}", flush=True)
    Ycv = np.concatenate([a for a, _ in res])
    Rcv = np.concatenate([b for _, b in res])
    near = (Ycv > -8.5) & (Ycv < -2.0)
    margin = [float(max(0.1, np.quantile(Rcv[near[:, j], j], quantile) + 0.05)) for j in range(4)]
    X, Y = table(rows)
    net, norm, final_loss = _fit(X, Y, hidden, steps, lr, seed)
    w = net.get_params()
    in_mean, in_std, out_mean, out_std = norm
    rec = {"format": "esp-proposer-2", "features": list(FEATURES), "outputs": list(OUTPUTS),
           "dims": net.dims, "params": [float(v) for v in w],
           "in_mean": in_mean.tolist(), "in_std": in_std.tolist(),
           "out_mean": out_mean.tolist(), "out_std": out_std.tolist(), "margin": margin,
           "cost": [0.0, 0.0, 0.0, 0.0, 0.0], "cost_unit": "us",
           "train": {"data": os.path.relpath(data_path, os.path.dirname(_HERE)), "data_sha256_16": _data_hash(data_path),
                     "rows": len(rows), "systems": len(systems), "steps": steps, "lr": lr, "seed": seed,
                     "hidden": list(hidden), "final_loss": final_loss,
                     "train_rmse": np.sqrt(np.mean((Y - _predict(net, norm, X)) ** 2, axis=0)).tolist(),
                     "cv_folds": folds, "cv_rmse": np.sqrt(np.mean(Rcv ** 2, axis=0)).tolist(),
                     "cv_quantile": quantile,
                     "cv_under_quantile": [float(np.quantile(Rcv[near[:, j], j], quantile)) for j in range(4)]}}
    net.close()
    return rec


# ---------------------------------------------------------------- cost model
def calibrate_cost(reps=30, seed=0):
    """Time one forces+energy+virial call over a sweep of (N, P, M) on the
    GPU and fit t = c0 + c1 N P^3 + c2 G log2 G + c3 N + c4 G (microseconds,
    non-negative least squares)."""
    import torch
    from scipy.optimize import nnls
    from . import synth
    rows = []
    for L, n_mol in ((3.0, 900), (4.5, 3000), (6.7, 10000), (9.0, 24000)):
        h, r, q = synth.water(n_mol, synth.cubic(L), config=6, seed=seed)
        xyz = torch.tensor(r, dtype=torch.float32, device="cuda")
        qq = torch.tensor(q, dtype=torch.float32, device="cuda")
        n = len(q)
        for delta in (1e-3, 1e-4, 1e-5, 1e-6):
            c = esp.c_from_delta(delta)
            D = int(np.ceil(-np.log10(delta) - 1e-9))
            for P, sigma in [(P, s) for P in (D, D + 1, D + 2) for s in (0.9, 1.3)]:
                M = _smooth(max(P, int(np.ceil(sigma * L * c / (np.pi * 0.9)))))
                plan = esp.Plan(h, n, delta, c_split=c, P=P, M=M)
                f = torch.empty((n, 3), dtype=torch.float32, device="cuda")
                out7 = torch.empty(7, dtype=torch.float64, device="cuda")
                for _ in range(5):
                    plan.forces(xyz, qq, f=f, out7=out7)
                t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                t0.record()
                for _ in range(reps):
                    plan.forces(xyz, qq, f=f, out7=out7)
                t1.record()
                torch.cuda.synchronize()
                us = t0.elapsed_time(t1) * 1e3 / reps
                G = float(M) ** 3
                rows.append((n, P, M, us, [1.0, n * P ** 3, G * np.log2(G), n, G]))
                plan.close()
                print(f"cost n={n} P={P} M={M}: {us:.1f} us", flush=True)
    A = np.array([r[4] for r in rows])
    t = np.array([r[3] for r in rows])
    scale = A.max(0)
    coef, _ = nnls(A / scale, t)
    coef = coef / scale
    pred = A @ coef
    return coef.tolist(), {"points": len(rows), "max_rel_dev": float(np.max(np.abs(pred - t) / t)),
                           "sweep": [[r[0], r[1], r[2], round(r[3], 2)] for r in rows]}


def _smooth(m):
    m = int(m)
    while True:
        k = m
        for p in (2, 3, 5):
            while k % p == 0:
                k //= p
        if k == 1:
            return m
        m += 1


# ---------------------------------------------------------------- registration
_registered = {}


def register(rec):
    """Create the network on the current device and register it with the planner."""
    net = Mlp(rec["dims"], seed=1)
    net.set_params(np.asarray(rec["params"], np.float32))
    p = esp.Proposer()
    p.mlp = net.handle.value
    for name in ("in_mean", "in_std", "out_mean", "out_std", "cost"):
        arr = getattr(p, name)
        for i, v in enumerate(rec[name]):
            arr[i] = float(v)
    for i, v in enumerate(rec["margin"]):
        p.margin[i] = float(v)
    st = esp.lib().esp_proposer_set(ctypes.byref(p))
    if st != esp.ESP_OK:
        raise esp.EspError(st, "esp_proposer_set rejected the weight record")
    old = _registered.pop("net", None)
    _registered["net"] = net
    _registered["rec"] = rec
    if old is not None:
        old.close()
    return net


def unregister():
    esp.lib().esp_proposer_set(None)
    net = _registered.pop("net", None)
    _registered.pop("rec", None)
    if net is not None:
        net.close()


def ensure_default():
    """Register the shipped weights once (raises if they are missing)."""
    if "net" in _registered:
        return _registered["rec"]
    if not os.path.exists(WEIGHTS_PATH):
        raise RuntimeError(f"{WEIGHTS_PATH} is missing: train it with `python -m paper_2601_00161_amd.learned`")
    with open(WEIGHTS_PATH) as f:
        rec = json.load(f)
    register(rec)
    return rec


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--data", required=True)
    tr.add_argument("--out", required=True)
    tr.add_argument("--steps", type=int, default=2000)
    tr.add_argument("--lr", type=float, default=3e-3)
    tr.add_argument("--hidden", default="16,16")
    co = sub.add_parser("cost")
    co.add_argument("--out", required=True)
    args = ap.parse_args()
    if args.cmd == "train":
        rec = train(args.data, hidden=tuple(int(v) for v in args.hidden.split(",")), steps=args.steps, lr=args.lr)
        if os.path.exists(args.out):
            with open(args.out) as f:
                old = json.load(f)
            rec["cost"], rec["cost_fit"] = old.get("cost", rec["cost"]), old.get("cost_fit")
    else:
        with open(args.out) as f:
            rec = json.load(f)
        rec["cost"], rec["cost_fit"] = calibrate_cost()
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
