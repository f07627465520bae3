"""Autotuner for the launch shape of a plan: the spreading tile edge, the
gather variant (per particle, or tile-staged potential in LDS) and the LDS
accumulator of the spreading (FP64, or 64-bit fixed point: always tried for
FP32 plans, for FP64 plans where tiles hold 128+ particles on average).

Each admissible candidate is timed on the GPU with the caller's own
particles (one esp_forces call = one step, HIP events over repeated calls)
and the fastest is kept.  Results are cached in a JSON file keyed by what
the choice depends on: precision, grid, window support, window degree class
and particle count (two significant digits).  Tuning never changes results
beyond the rounding of the plan's precision: every candidate computes the
same sums, reassociated (and, in fixed point, each term rounded to at most
2^-61 of its tile's charge bound).

    plan, info = autotune.tuned_plan(h, n, tol, xyz, q, cache="tune.json", precision="fp32")

Batches (many replicas, one launch per stage) are tuned on the batch itself:
tune_batch times the whole batched step for each candidate tile edge of
each window-support group.
"""
from __future__ import annotations

import json
import math
import os

from . import esp

TILES = (4, 5, 6, 8, 10, 12)
GATHERS = ("particle", "tile", "lane")
ACCUMS = ("fp64", "fixed")
FIXED_MIN_PER_TILE = 128          # FP64 plans: fixed point is tried from this many particles per tile
DEFAULT_CACHE = os.environ.get("ESP_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                                  "esp_mi355x_autotune.json"))


def _key(params):
    n = params["n"]
    n2 = int(round(n, -max(0, int(math.floor(math.log10(n))) - 1)))
    cls = 8 if params["window_degree"] <= 8 else (12 if params["window_degree"] <= 12 else 16)
    return (f"{'fp32' if params['precision'] == 0 else 'fp64'}:M{params['M'][0]}x{params['M'][1]}x{params['M'][2]}"
            f":P{params['P']}:W{cls}:N{n2}")


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _save(path, data):
    if not path:
        return
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_step(plan, xyz, q, reps=20, warmup=3):
    """Microseconds per esp_forces call (HIP events around `reps` calls)."""
    import torch
    f, out = plan.forces(xyz, q)
    for _ in range(warmup):
        plan.forces(xyz, q, f=f, out7=out)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.forces(xyz, q, f=f, out7=out)
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / reps


def tune(h, n, tol, xyz, q, reps=20, tiles=TILES, gathers=GATHERS, accums=ACCUMS, **opts):
    """Time every admissible (tile, gather, accumulator) choice; returns
    {"tile", "gather", "accum", "us", "table"} (table keys "tile:gather" for
    the FP64 accumulator, "tile:gather:fixed" for fixed point)."""
    table = {}
    best = None
    for t in tiles:
        for g in gathers:
            for a in accums:
                try:
                    plan = esp.Plan(h, n, tol, tile=t, gather=g, spread_accum=a, **opts)
                except esp.EspError:
                    continue                  # not admissible for this grid (LDS, tile count)
                if (a == "fixed" and plan.params["precision"] == 1
                        and n < FIXED_MIN_PER_TILE * plan.params["ntiles"]):
                    plan.close()              # FP64, sparse tiles: fixed point is slower (measured)
                    continue
                us = time_step(plan, xyz, q, reps=reps)
                plan.close()
                table[f"{t}:{g}" + (":fixed" if a == "fixed" else "")] = round(us, 2)
                if best is None or us < best[3]:
                    best = (t, g, a, us)
    if best is None:
        raise RuntimeError("no admissible launch shape")
    return {"tile": best[0], "gather": best[1], "accum": best[2], "us": round(best[3], 2), "table": table}


def tuned_plan(h, n, tol, xyz, q, cache=DEFAULT_CACHE, retune=False, tiles=TILES, gathers=GATHERS, **opts):
    """A plan with the cached (or freshly tuned) launch shape for this problem
    (candidates: the given tile edges and gather variants)."""
    probe = esp.Plan(h, n, tol, **opts)
    key = _key(probe.params)
    probe.close()
    data = _load(cache)
    if retune or key not in data:
        data[key] = tune(h, n, tol, xyz, q, tiles=tiles, gathers=gathers, **opts)
        _save(cache, data)
    rec = data[key]
    plan = esp.Plan(h, n, tol, tile=rec["tile"], gather=rec["gather"], spread_accum=rec.get("accum", "fp64"),
                    **opts)
    return plan, dict(rec, key=key)


def _batch_ms(batch, xyz, q, reps=10, windows=3):
    """Median over `windows` of the milliseconds per batched esp_batch_forces
    call (HIP events around `reps` graph-replayed calls)."""
    import torch
    f, out = batch.forces(xyz, q)
    for _ in range(3):
        batch.forces(xyz, q, f=f, out7=out)
    ms = []
    for _ in range(windows):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            batch.forces(xyz, q, f=f, out7=out)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b) / reps)
    return sorted(ms)[len(ms) // 2]


def _batch_key(params):
    import hashlib
    txt = ";".join(_key(p) for p in params)
    return "batch:" + hashlib.sha256(txt.encode()).hexdigest()[:16]


def tune_batch(cells, ns, tols, xyz, q, cache=DEFAULT_CACHE, retune=False, tiles=TILES, **opts):
    """Spreading tile edges for esp.Batch, chosen by timing the batch itself.

    The batch spreads and gathers in one launch per window support P, so the
    tile edge is chosen per P group: starting from each plan's own rule, every
    group tries every admissible edge for all its replicas (the other groups
    at their current choice) and keeps the fastest batch step; one pass over
    the groups.  Returns {"tiles": per replica (0 = the plan's rule),
    "groups": {P: edge}, "default_ms", "ms", "key"}; cached like tuned_plan.
    Results of a tuned batch equal the default batch's up to reassociation
    (the tile edge only changes which workgroup adds which terms)."""
    probe = esp.Batch(cells, ns, tols, graph=True, **opts)
    key = _batch_key(probe.params)
    Ps = [p["P"] for p in probe.params]
    data = _load(cache)
    if not retune and key in data:
        probe.close()
        return dict(data[key], key=key)
    base = _batch_ms(probe, xyz, q)
    probe.close()
    current = [0] * len(ns)
    best = base
    groups = {}
    for P in sorted(set(Ps)):
        idx = [i for i, p in enumerate(Ps) if p == P]
        pick = 0
        for t in tiles:
            trial = list(current)
            for i in idx:
                trial[i] = t
            try:
                b = esp.Batch(cells, ns, tols, tiles=trial, graph=True, **opts)
            except esp.EspError:
                continue                      # not admissible for some replica of the group
            ms = _batch_ms(b, xyz, q)
            b.close()
            if ms < best:
                best, pick = ms, t
        for i in idx:
            current[i] = pick
        groups[str(P)] = pick
    rec = {"tiles": current, "groups": groups, "default_ms": round(base, 4), "ms": round(best, 4)}
    data[key] = rec
    _save(cache, data)
    return dict(rec, key=key)
