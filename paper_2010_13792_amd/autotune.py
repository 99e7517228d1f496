"""Autotuner for the launch options of a recorded call sequence.

``tune`` times a user-supplied ``run(params) -> milliseconds`` for every
candidate parameter set (median of ``reps`` runs after one warm-up), keeps
the fastest, and stores the choice in a JSON cache keyed by the device name
and a caller-chosen workload signature, so later runs on the same device and
workload shape reuse it without re-timing.
"""
from __future__ import annotations

import itertools
import json
import os
import statistics

import torch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "adaptgrav", "autotune.json")


def _cache_path():
    return os.environ.get("AG_AUTOTUNE_CACHE", DEFAULT_CACHE)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def grid(**axes):
    """Cartesian product of option axes as a list of dicts."""
    keys = list(axes)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(axes[k] for k in keys))]


def tune(run, candidates, signature: str, reps: int = 3, use_cache: bool = True):
    """Return (best_params, table) where table maps str(params) -> median ms."""
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    key = f"{dev}|{signature}"
    path = _cache_path()
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        return cache[key]["best"], cache[key]["table"]
    table = {}
    best, best_ms = None, float("inf")
    for p in candidates:
        run(p)   # warm-up (allocations, code loading)
        ms = statistics.median(run(p) for _ in range(reps))
        table[json.dumps(p, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = p, ms
    if use_cache:
        cache[key] = {"best": best, "table": table}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best, table
