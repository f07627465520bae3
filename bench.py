#!/usr/bin/env python3
"""Throughput of the ESP reciprocal-space path (energy + forces + virial).

One step = one esp_forces call (cell sort, spreading, forward FFT, scaling and
reduction, potential, inverse FFT, gather, finalisation) for all N particles
of the workload, inputs already resident in device memory.

Workload (default): bulk-water-shaped system, 10,000 rigid 3-site triplets in
a cubic 6.7 nm cell (N = 30,000), tolerance 1e-5, seeded synthetic input.
The headline value is the FP32 path with learned parameters (the
registered proposer; the analytic rule if it declines); the FP32 path with
the analytic rule and the plain FP64 path (analytic parameters) are timed
beside it on the same input.  The CPU leg runs the oracle: the baseline
timing, parity at identical parameters, and the error of every GPU result
against an exact reference.

Prints ONE JSON line.  Its "roofline" object rates the dominant kernel by
algorithmic bytes per launch (stage_bytes below: e.g. spreading reads 16 B
per particle record and writes 4 B per grid point) over its live launch
time, against the 8 TB/s HBM peak, next to the HBM traffic measured by the
FETCH_SIZE / WRITE_SIZE counter passes recorded under profiles/.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per launch (per particle / per grid point) of each stage;
# r = bytes of a real, N particles, G = M1 M2 M3 grid points, S = complex
# half-spectrum entries (M1/2+1) M2 M3.
def stage_bytes(stage, N, G, S, r):
    rec = 16 if r == 4 else 32                     # sorted particle record
    c = 2 * r
    return {
        "bin": N * (4 * r + rec + 8),               # xyz, q in; record, key, rank out
        "scatter": N * (rec + 8 + rec + 4),         # record, key, rank in; record, perm out
        "spread": N * rec + G * r,                  # sorted records in, grid out
        "fft_xy": G * r + S * c,                    # real grid in, half spectrum out
        "fft_z": 2 * S * c,                         # spectrum in and out
        "fft_xy_inv": S * c + G * r,
        "gather": N * (rec + 4 + 3 * r) + G * r,    # records, perm in; forces out; phi in
    }[stage]


def run_plan(plan, xyz, q, steps, warmup, torch):
    f, out7 = plan.forces(xyz, q)
    for _ in range(warmup):
        plan.forces(xyz, q, f=f, out7=out7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.forces(xyz, q, f=f, out7=out7)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.check()
    return dt, f, out7


KERNEL_SOURCES = {
    "spread": ("esp_stencil.hip", "esp_common.h", "esp_device.h"),
    "gather": ("esp_stencil.hip", "esp_common.h", "esp_device.h"),
    "bin": ("esp_kernels.hip", "esp_common.h", "esp_device.h"),
    "scatter": ("esp_kernels.hip", "esp_common.h", "esp_device.h"),
    "fft_xy": ("esp_kernels.hip", "esp_common.h", "esp_device.h"),
    "fft_z": ("esp_kernels.hip", "esp_common.h", "esp_device.h"),
    "fft_xy_inv": ("esp_kernels.hip", "esp_common.h", "esp_device.h"),
}


def sources_sha(kernel):
    import hashlib
    hsh = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2601_00161_amd", "csrc", name), "rb") as f:
            hsh.update(f.read())
    return hsh.hexdigest()[:16]


def measured_traffic(kernel, workload_key):
    """HBM bytes per launch from the committed counter summary, or None when
    there is none for this kernel and workload or the kernel's sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_water30k.md")
    if not os.path.exists(path):
        return None
    want = sources_sha(kernel)
    for line in open(path):
        if line.startswith("TRAFFIC "):
            kv = dict(item.split("=", 1) for item in line.split()[1:])
            if kv.get("kernel") == kernel and kv.get("workload") == workload_key and kv.get("sources") == want:
                return float(kv["bytes_per_launch"])
    return None


def oracle_leg(h, r32, q32, plans, headline):
    """CPU side (the oracle, FP64): baseline timing, parity of each GPU plan at
    identical parameters, and the headline's error against an exact reference
    (the oracle's ESP at Delta = 1e-11, P = 12, whose CPU tests pin it to
    classical Ewald) with the oracle's real-space part added."""
    from oracle import esp_direct, esp_grid
    from oracle.pswf import c_from_tol
    r64, q64 = r32.astype(np.float64), q32.astype(np.float64)
    N = len(q64)

    def gp(prm):
        return esp_grid.GridParams(prm["c_split"], prm["c_spread"], prm["P"], tuple(prm["M"]), prm["rc"])

    def w6(W):
        return np.array([W[0, 0], W[1, 1], W[2, 2], W[0, 1], W[0, 2], W[1, 2]])

    out = {"parity_vs_oracle": {}}
    refs = {}
    for name, (plan, f, o) in plans.items():
        prm = plan.params
        key = (prm["c_split"], prm["P"], tuple(prm["M"]), prm["force"])
        if key not in refs:
            refs[key] = (esp_grid.esp_grid_ik if prm["force"] == 1 else esp_grid.esp_grid)(h, r64, q64, gp(prm))
        ref = refs[key]
        fo, oo = f.cpu().numpy().astype(np.float64), o.cpu().numpy()
        out["parity_vs_oracle"][name] = {
            "energy": float(abs(oo[0] - ref.energy) / abs(ref.energy)),
            "virial": float(np.linalg.norm(oo[1:] - w6(ref.virial)) / np.linalg.norm(w6(ref.virial))),
            "forces_rms": float(np.sqrt(np.sum((fo - ref.forces) ** 2) / np.sum(ref.forces ** 2)))}

    # CPU baseline: the oracle's gridded ESP at the FP64 plan's parameters
    p64 = plans["fp64_analytic"][0].params
    reps, t0 = 0, time.perf_counter()
    while reps < 1 or time.perf_counter() - t0 < 10.0:
        esp_grid.esp_grid(h, r64, q64, gp(p64))
        reps += 1
    tc = (time.perf_counter() - t0) / reps
    out["cpu_baseline"] = {
        "value": N / tc / 1e6, "unit": "M particle-steps/s", "cores": 1, "kind": "oracle",
        "sample": f"{reps} full steps of the oracle's gridded FP64 ESP (numpy, single thread) on the same "
                  f"N={N} workload at the FP64 plan's parameters; host has {len(os.sched_getaffinity(0))} cores"}

    # exact reference of the total Coulomb energy, virial and forces
    c_ref = c_from_tol(1e-11)
    M_ref = int(np.ceil(1.07 * max(np.linalg.norm(h, axis=0)) * c_ref / (np.pi * 0.9)))
    M_ref += M_ref % 2
    ex_F = esp_grid.esp_grid(h, r64, q64, esp_grid.GridParams(c_ref, c_ref, 12, (M_ref,) * 3, 0.9))
    U_N, W_N, F_N = esp_direct.real_space(h, r64, q64, c_ref, 0.9)
    E_ex, W_ex, F_ex = ex_F.energy + U_N, ex_F.virial + W_N, ex_F.forces + F_N
    acc = {}
    for name, (plan, f, o) in plans.items():
        prm = plan.params
        u_n, w_n, f_n = esp_direct.real_space(h, r64, q64, prm["c_split"], prm["rc"])
        oo = o.cpu().numpy()
        W = np.array([[oo[1], oo[4], oo[5]], [oo[4], oo[2], oo[6]], [oo[5], oo[6], oo[3]]]) + w_n
        F = f.cpu().numpy().astype(np.float64) + f_n
        dg = [(W[a, a] - W_ex[a, a]) for a in range(3)]
        od = [(W[a, b] - W_ex[a, b]) for a, b in ((0, 1), (0, 2), (1, 2))]
        acc[name] = {
            "energy": float(abs(oo[0] + u_n - E_ex) / abs(E_ex)),
            "pressure_diag": float(np.linalg.norm(dg) / np.linalg.norm(np.diag(W_ex))),
            "pressure_offdiag": float(np.linalg.norm(od) / np.linalg.norm([W_ex[0, 1], W_ex[0, 2], W_ex[1, 2]])),
            "forces_rms": float(np.sqrt(np.sum((F - F_ex) ** 2) / np.sum(F_ex ** 2)))}
    out["accuracy_vs_exact"] = acc
    out["accuracy_reference"] = (f"total Coulomb (real + reciprocal) from the oracle's ESP at Delta=1e-11, P=12, "
                                 f"M={M_ref}^3; each GPU result gets the oracle's real-space part at its own c")
    return out


def batch_throughput(torch, dev, steps=20):
    """The 64-replica batch (N in [2,000, 60,000], per-replica tol in
    {1e-3 ... 1e-6}, FP32, learned parameters): particle-steps per second of
    one graph-replayed call per step, next to the same replicas run as 64
    single-plan calls."""
    from paper_2601_00161_amd import synth
    from paper_2601_00161_amd.esp import Batch, Plan
    reps = synth.replicas()
    cells = [x[0] for x in reps]
    ns = [len(x[2]) for x in reps]
    tols = [x[3] for x in reps]
    xyz = torch.tensor(np.concatenate([x[1] for x in reps]), dtype=torch.float32, device=dev)
    q = torch.tensor(np.concatenate([x[2] for x in reps]), dtype=torch.float32, device=dev)
    b = Batch(cells, ns, tols, graph=True, params="learned")
    f, out = b.forces(xyz, q)
    for _ in range(3):
        b.forces(xyz, q, f=f, out7=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.forces(xyz, q, f=f, out7=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    b.check()
    launches = b.num_launches(True)
    b.close()
    # the same replicas as single plans, one after the other
    plans = [Plan(c, n, t, params="learned") for c, n, t in zip(cells, ns, tols)]
    offs = np.concatenate([[0], np.cumsum(ns)])
    views = [(xyz[offs[k]:offs[k + 1]], q[offs[k]:offs[k + 1]]) for k in range(len(ns))]
    outs = [p.forces(*v) for p, v in zip(plans, views)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for p, v, (fo, oo) in zip(plans, views, outs):
            p.forces(*v, f=fo, out7=oo)
    torch.cuda.synchronize()
    ds = (time.perf_counter() - t0) / steps
    for p in plans:
        p.close()
    total = int(sum(ns))
    return {"replicas": len(ns), "particles": total, "launches_per_step": launches,
            "ms_per_step": dt * 1e3, "value": total / dt / 1e6, "unit": "M particle-steps/s",
            "single_plans_ms_per_step": ds * 1e3, "speedup_vs_single_plans": ds / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--tile", type=int, default=0, help="spreading tile edge (0 = plan default)")
    ap.add_argument("--params", default="learned", choices=["learned", "analytic"],
                    help="parameter source of the FP32 headline plan")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner (plan defaults)")
    ap.add_argument("--gather", default="auto", choices=["auto", "particle", "tile"],
                    help="gather variant when the launch shape is given (--tile or --no-tune)")
    ap.add_argument("--counters-only", action="store_true",
                    help="run only the headline plan (at --tile / --gather) and the near part, for counter passes")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-replica batch measurement")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first run 5 plain device copies of MIB MiB (float32), the known-size "
                         "kernel that calibrates the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); the slab decomposition "
              "over several GPUs is designed but not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2601_00161_amd import synth
    from paper_2601_00161_amd.esp import PARAMS, Plan

    dev = torch.device("cuda:0")
    if args.copy_calib > 0:
        n = args.copy_calib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"copy calibration: 5 copies of {args.copy_calib} MiB", file=sys.stderr, flush=True)
        del a, b
    h, r, q = synth.config2(args.seed)
    N = len(q)
    r32, q32 = r.astype(np.float32), q.astype(np.float32)
    x32, c32 = torch.from_numpy(r32).to(dev), torch.from_numpy(q32).to(dev)
    x64, c64 = torch.from_numpy(r32.astype(np.float64)).to(dev), torch.from_numpy(q32.astype(np.float64)).to(dev)

    if args.counters_only:
        # one plan at a fixed launch shape, so that per-kernel counters are not
        # mixed with the autotuner's trial shapes
        p = Plan(h, N, args.tol, precision="fp32", params=args.params, tile=args.tile, gather=args.gather)
        f, o = p.forces(x32, c32)
        fn, on = p.real_space(x32, c32)
        for _ in range(args.warmup + args.steps):
            p.forces(x32, c32, f=f, out7=o)
            p.real_space(x32, c32, f=fn, out7=on)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "tile": p.params["tile"], "gather_tiled": p.params["gather_tiled"],
                          "P": p.params["P"], "M": p.params["M"], "launches": args.warmup + args.steps}))
        p.close()
        return

    import tempfile
    from paper_2601_00161_amd import autotune
    tune_dir = tempfile.TemporaryDirectory()

    def make_plan(precision, params, xyz, q):
        """A plan with the autotuned launch shape (tile edge, gather variant)."""
        if args.no_tune or args.tile:
            return Plan(h, N, args.tol, precision=precision, params=params, tile=args.tile, gather=args.gather), None
        return autotune.tuned_plan(h, N, args.tol, xyz, q, cache=os.path.join(tune_dir.name, "tune.json"),
                                   precision=precision, params=params)

    # ---- FP32 headline path (learned parameters, autotuned launch shape) ------------
    p32, tuned = make_plan("fp32", args.params, x32, c32)
    for _ in range(10):                      # first launches load code objects
        p32.forces(x32, c32)
    torch.cuda.synchronize()
    # pre-pass: every stage timed once per step to find the dominant kernel
    p32.profile(["bin", "scatter", "spread", "fft_xy", "fft_z", "fft_xy_inv", "gather"], 64)
    for _ in range(32):
        p32.forces(x32, c32)
    stages = p32.profile_read()
    dominant = max(stages, key=lambda s: stages[s][0] / stages[s][1])
    # timed region, with events around every 8th launch of the dominant kernel
    p32.profile([dominant], args.steps + args.warmup + 2, stride=8)
    dt32, f32, o32 = run_plan(p32, x32, c32, args.steps, args.warmup, torch)
    dom_ms, dom_n = p32.profile_read()[dominant]
    p32.profile([], 0)

    # ---- FP32 with the analytic rule (the proposer's gain) ---------------------
    pa, tuned_a = make_plan("fp32", "analytic", x32, c32)
    dta, fa, oa = run_plan(pa, x32, c32, args.steps, args.warmup, torch)

    # ---- FP32 with ik-differentiated forces (momentum-conserving option) ------------
    pik = Plan(h, N, args.tol, precision="fp32", params=args.params, force="ik", tile=p32.params["tile"][0])
    dtik, fik, oik = run_plan(pik, x32, c32, args.steps, args.warmup, torch)

    # ---- FP32 per-particle virial (local pressure) ----------------------------------
    ploc = Plan(h, N, args.tol, precision="fp32", params=args.params, local_virial=True,
                tile=p32.params["tile"][0])
    w6, o_loc = ploc.local_virial(x32, c32, out7=torch.empty(7, dtype=torch.float64, device=dev))
    for _ in range(args.warmup):
        ploc.local_virial(x32, c32, w6=w6, out7=o_loc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ploc.local_virial(x32, c32, w6=w6, out7=o_loc)
    torch.cuda.synchronize()
    dtloc = time.perf_counter() - t0
    loc_sum_err = float(np.max(np.abs(w6.double().sum(0).cpu().numpy() - o_loc.cpu().numpy()[1:]))
                        / np.max(np.abs(o_loc.cpu().numpy()[1:])))
    ploc.close()

    # ---- real-space (near) part, and the total Coulomb step (Fourier forces plus
    # near forces accumulated in place) on the headline plan --------------------------
    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # pressure-only path (energy and virial from one forward FFT, no forces)
    o_ev = torch.empty(7, dtype=torch.float64, device=dev)
    dt_ev = timed(lambda: p32.energy_virial(x32, c32, out7=o_ev))

    f_near = torch.empty_like(f32)
    o_near = torch.empty(7, dtype=torch.float64, device=dev)
    dt_near = timed(lambda: p32.real_space(x32, c32, f=f_near, out7=o_near))
    f_tot = torch.empty_like(f32)
    o_tot = torch.empty(7, dtype=torch.float64, device=dev)

    def total_step():
        p32.forces(x32, c32, f=f_tot, out7=o_tot)
        p32.real_space(x32, c32, f=f_tot, out7=o_near, accumulate=True)
    dt_tot = timed(total_step)
    # the same total with the near part on a second stream beside the Fourier part
    dt_ovl = timed(lambda: p32.coulomb(x32, c32, f=f_tot, out7=o_tot))

    # ---- plain FP64 path, analytic parameters -------------------------------------
    p64, tuned_64 = make_plan("fp64", "analytic", x64, c64)
    dt64, f64, o64 = run_plan(p64, x64, c64, args.steps, args.warmup, torch)

    f64_near = torch.empty_like(f64)
    o64_near = torch.empty(7, dtype=torch.float64, device=dev)
    dt64_near = timed(lambda: p64.real_space(x64, c64, f=f64_near, out7=o64_near))

    batch = None if args.no_batch else batch_throughput(torch, dev)

    cpu = None
    extra = {}
    if not args.no_cpu:
        extra = oracle_leg(h, r32, q32, {"fp32_headline": (p32, f32, o32), "fp32_analytic": (pa, fa, oa),
                                         "fp64_analytic": (p64, f64, o64), "fp32_ik": (pik, fik, oik)},
                           "fp32_headline")
        cpu = extra.pop("cpu_baseline")

    prm = p32.params
    G = prm["M"][0] * prm["M"][1] * prm["M"][2]
    S = (prm["M"][0] // 2 + 1) * prm["M"][1] * prm["M"][2]
    avg_s = dom_ms / dom_n / 1e3
    bytes_dom = stage_bytes(dominant, N, G, S, 4)
    achieved = bytes_dom / avg_s / 1e9
    workload_key = (f"water30k_tol{args.tol:g}_P{prm['P']}_M{prm['M'][0]}x{prm['M'][1]}x{prm['M'][2]}"
                    f"_T{prm['tile'][0]}_{'gtile' if prm['gather_tiled'] else 'gpart'}"
                    f"{'_fixed' if prm['spread_fixed'] else ''}")
    traffic = measured_traffic(dominant, workload_key)
    value = N * args.steps / dt32 / 1e6
    v64 = N * args.steps / dt64 / 1e6
    va = N * args.steps / dta / 1e6
    src = {v: k for k, v in PARAMS.items()}[prm["params_source"]]

    def brief(p):
        return {"source": {v: k for k, v in PARAMS.items()}[p.params["params_source"]],
                "delta": p.params["delta"], "c": p.params["c_split"], "P": p.params["P"], "M": p.params["M"],
                "tile": p.params["tile"], "gather_tiled": p.params["gather_tiled"]}

    line = {
        "metric": "M particle-steps/s (E+F+virial) at 1e-5 rel err: FP32+learned vs plain FP64",
        "value": round(value, 3),
        "unit": "M particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "bulk-water-shaped, 10,000 rigid 3-site triplets, cubic 6.7 nm, N=30000, tol 1e-5",
                   "seed": args.seed, "params": src, "delta": prm["delta"], "c": prm["c_split"], "P": prm["P"],
                   "M": prm["M"], "rc": prm["rc"], "tile": prm["tile"], "gather_tiled": prm["gather_tiled"],
                   "autotune": tuned,
                   "predicted_log10_err": prm["predicted_log10_err"] if src == "learned" else None},
        "fp64_baseline": {"value": round(v64, 3), "ms_per_step": dt64 / args.steps * 1e3, **brief(p64)},
        "speedup_vs_fp64": value / v64,
        "fp32_analytic": {"value": round(va, 3), "ms_per_step": dta / args.steps * 1e3, **brief(pa)},
        "learned_gain_vs_analytic": value / va,
        "batch_64_replicas": batch,
        "local_virial_fp32": {"value": round(N * args.steps / dtloc / 1e6, 3), "unit": "M particle-steps/s",
                              "ms_per_step": dtloc / args.steps * 1e3, "shares_sum_rel_err": loc_sum_err},
        "ik_forces_fp32": {"value": round(N * args.steps / dtik / 1e6, 3), "ms_per_step": dtik / args.steps * 1e3,
                           "net_force_over_rms": float(np.linalg.norm(fik.double().sum(0).cpu().numpy())
                                                       / np.sqrt(np.sum(fik.double().cpu().numpy() ** 2)))},
        "energy_virial_fp32": {"value": round(N * args.steps / dt_ev / 1e6, 3), "unit": "M particle-steps/s",
                               "ms_per_step": dt_ev / args.steps * 1e3},
        "real_space": {"unit": "M particle-steps/s", "cells": prm["real_cells"], "rc": prm["rc"],
                       "fp32": {"value": round(N * args.steps / dt_near / 1e6, 3),
                                "ms_per_step": dt_near / args.steps * 1e3},
                       "fp64": {"value": round(N * args.steps / dt64_near / 1e6, 3),
                                "ms_per_step": dt64_near / args.steps * 1e3},
                       "total_coulomb_fp32": {"value": round(N * args.steps / dt_tot / 1e6, 3),
                                              "ms_per_step": dt_tot / args.steps * 1e3},
                       "total_coulomb_overlapped_fp32": {"value": round(N * args.steps / dt_ovl / 1e6, 3),
                                                         "ms_per_step": dt_ovl / args.steps * 1e3}},
        **extra,
        "stage_ms_fp32": {k: v[0] / v[1] for k, v in stages.items()},
        "roofline": {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_dom, "avg_launch_us": avg_s * 1e6, "workload_key": workload_key},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
