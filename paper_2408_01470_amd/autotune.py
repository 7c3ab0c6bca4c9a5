"""Autotuner of the annealing kernel's launch shape.

Candidates are (waves per workgroup, register budget in waves per SIMD).
Each is timed on a short slice of the real calibration (a few levels, HIP
events around every level kernel on the launch stream); the fastest is
cached in a JSON file keyed by the problem's shape:
(architecture, model, formula, residual, quotes bucket, chains bucket,
instances bucket).  The cache path is $SABR_AUTOTUNE_CACHE or
~/.cache/sabr_autotune.json.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

CANDIDATES = ((1, 1), (2, 1), (4, 1), (1, 3), (2, 3), (4, 3), (2, 4), (4, 4), (6, 4), (8, 1),
              (8, 3), (8, 4))


def cache_path():
    return os.environ.get("SABR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "sabr_autotune.json"))


def _bucket(v):
    return int(2 ** int(np.ceil(np.log2(max(int(v), 1)))))


def shape_key(plan, chains):
    ch = np.broadcast_to(np.asarray(chains), (plan.n_inst,))
    arch = torch.cuda.get_device_properties(plan.device).gcnArchName.split(":")[0]
    return (f"{arch}|m{plan.model}|f{plan.formula}|r{plan.residual}|q{_bucket(plan.max_q)}"
            f"|c{_bucket(ch.max())}|i{_bucket(plan.n_inst)}")


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(plan, chains):
    hit = _load().get(shape_key(plan, chains))
    return (hit["waves"], hit["occupancy"]) if hit else None


def tune(plan, chains, lb, ub, n_steps, levels=4, candidates=CANDIDATES, store=True):
    """Time each candidate on `levels` levels (the first is a warm-up) and
    return {"waves", "occupancy", "level_ms", "all"}."""
    stream = torch.cuda.current_stream()
    results = []
    ws = None
    for waves, occ in candidates:
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * levels)]
        for e in evs:
            e.record(stream)
        r = plan.sa(chains, lb, ub, T0=1.0, cool=0.5, n_levels=levels, n_steps=n_steps, seed=1,
                    trace=False, waves=waves, occupancy=occ, level_events=evs, workspace=ws)
        ws = r["workspace"]
        torch.cuda.synchronize()
        ms = [evs[2 * l].elapsed_time(evs[2 * l + 1]) for l in range(1, levels)]
        results.append(dict(waves=waves, occupancy=occ, level_ms=float(np.mean(ms))))
    best = min(results, key=lambda d: d["level_ms"])
    out = dict(best, all=results)
    if store:
        cache = _load()
        cache[shape_key(plan, chains)] = dict(waves=best["waves"], occupancy=best["occupancy"],
                                              level_ms=best["level_ms"])
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return out
