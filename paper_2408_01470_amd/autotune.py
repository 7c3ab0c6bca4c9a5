"""Autotuner of the annealing kernel's launch shape.

Candidates are (waves per workgroup, register budget in waves per SIMD),
optionally with a third entry, the waves per chain (a chain's quotes split
over the waves of its own workgroup; split_candidates proposes them when
the chains alone leave most of the chip's SIMDs idle), and a fourth, the
chains per wave (two: one per half-wave, GLOBAL4 only; pair_candidates
proposes them when the chains fill the chip many times over).  Each is timed on a
short slice of the real calibration (a few levels, HIP events around every
level kernel on the launch stream); the fastest is cached in a JSON file
keyed by the problem's shape:
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


def split_candidates(plan, chains, simds=1024):
    """(waves, occupancy, waves per chain) shapes for few chains of many
    quotes: k = 2, 4, 8 waves per chain, each at most the chain's blocks of
    64 quotes, when all chains together fill fewer than `simds` waves."""
    total = int(np.sum(np.broadcast_to(np.asarray(chains), (plan.n_inst,))))
    blocks = -(-int(plan.max_q) // 64)
    if total >= simds or blocks < 2:
        return ()
    return tuple((k, occ, k) for k in (2, 4, 8) if k <= blocks for occ in (1, 3))


def pair_candidates(plan, chains, simds=1024):
    """(waves, occupancy, 1, 2) shapes: two chains per wave, one per half
    (GLOBAL4 only), when the chains fill every SIMD twice over even paired."""
    total = int(np.sum(np.broadcast_to(np.asarray(chains), (plan.n_inst,))))
    if plan.model != 0 or total < 4 * simds:
        return ()
    return tuple((w, occ, 1, 2) for w in (4, 8) for occ in (1, 3, 4))


def lookup(plan, chains):
    hit = _load().get(shape_key(plan, chains))
    return ((hit["waves"], hit["occupancy"], hit.get("waves_per_chain", 1),
             hit.get("chains_per_wave", 1)) if hit else None)


def tune(plan, chains, lb, ub, n_steps, levels=4, candidates=CANDIDATES, store=True):
    """Time each candidate on `levels` levels (the first is a warm-up) and
    return {"waves", "occupancy", "waves_per_chain", "chains_per_wave",
    "level_ms", "all"}."""
    stream = torch.cuda.current_stream()
    results = []
    ws = None
    for cand in candidates:
        waves, occ = cand[0], cand[1]
        wpc = cand[2] if len(cand) > 2 else 1
        cpw = cand[3] if len(cand) > 3 else 1
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 * levels)]
        for e in evs:
            e.record(stream)
        r = plan.sa(chains, lb, ub, T0=1.0, cool=0.5, n_levels=levels, n_steps=n_steps, seed=1,
                    trace=False, waves=waves, occupancy=occ, waves_per_chain=wpc,
                    chains_per_wave=cpw, level_events=evs, workspace=ws)
        ws = r["workspace"]
        torch.cuda.synchronize()
        ms = [evs[2 * l].elapsed_time(evs[2 * l + 1]) for l in range(1, levels)]
        results.append(dict(waves=waves, occupancy=occ, waves_per_chain=wpc,
                            chains_per_wave=cpw, level_ms=float(np.mean(ms))))
    best = min(results, key=lambda d: d["level_ms"])
    out = dict(best, all=results)
    if store:
        cache = _load()
        cache[shape_key(plan, chains)] = dict(waves=best["waves"], occupancy=best["occupancy"],
                                              waves_per_chain=best["waves_per_chain"],
                                              chains_per_wave=best["chains_per_wave"],
                                              level_ms=best["level_ms"])
        path = cache_path()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return out
