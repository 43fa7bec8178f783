"""Autotuning of batched launches, with a persistent tuning cache.

The timing loop runs in the library (boys_autotune: each candidate is built into a plan
and replayed with HIP events).  This module chooses the candidate set, keys the result by
device, library build and a coarse signature of the batch, and keeps it in a JSON cache
(``$BOYS_TUNING_FILE``, default ``~/.cache/paper_2504_07637_amd/tuning.json``).

Tunable choices (the per-argument work is one sequential chain, so a lane always owns
whole arguments): the schedule (persistent waves with work counters, one workgroup per
tile, or one wave per tile), the workgroup size, the arguments per lane (tile = block x 1,
2 or 4 for one workgroup per tile, 64 x 4 for one wave per tile and for the persistent
waves, with the store-bound arrays optionally in a launch of their own at one argument
per lane), the tile order (longest first, array by array, or grouped by class) and, for
the persistent schedule, the number of workgroups per compute unit.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

from . import _lib

CANDIDATES = (
    [{"schedule": 1, "block": b, "tile": b * k, "grid_per_cu": 1, "order": o}
     for o in (1, 2, 0) for b in (128, 256) for k in (1, 2, 4)]
    + [{"schedule": 0, "block": 256, "tile": 256, "grid_per_cu": g, "order": o}
       for o in (1, 0) for g in (4, 8)]
    + [{"schedule": 2, "block": b, "tile": 256, "grid_per_cu": 1, "order": o}
       for o in (1, 2) for b in (128, 256)]
    + [{"schedule": 2, "block": 256, "tile": 256, "grid_per_cu": 1, "order": 1, "split_nmax": k}
       for k in (8, 10, 12)]
)


def cache_path() -> str:
    p = os.environ.get("BOYS_TUNING_FILE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2504_07637_amd", "tuning.json")


def _lib_hash() -> str:
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def signature(lengths, n_maxs, precisions) -> str:
    """Coarse shape class of a batch: counts and sizes in powers of two."""
    total = sum(lengths)
    mean_len = total / max(1, len(lengths))
    fp32 = sum(1 for p in precisions if p in (1, "fp32", "float32", "mixed"))
    return (f"count2^{int(math.log2(max(1, len(lengths))))}"
            f"-len2^{int(math.log2(max(1.0, mean_len)))}"
            f"-nmax{max(n_maxs) if n_maxs else 0}"
            f"-fp32frac{round(fp32 / max(1, len(lengths)), 1)}")


def _device_key(torch, device) -> str:
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch}/{props.multi_processor_count}cu"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned(xs, n_maxs, precisions, candidates=CANDIDATES, warmup=12, reps=10, refresh=False):
    """The best tuning for this batch: from the cache, or measured now and cached.

    Each candidate is a fresh plan; a fresh plan runs slower for about its first dozen
    replays (measured), hence the warm-up before the timed replays.

    Returns (tuning dict, info dict with the key, whether it was cached and the times)."""
    import torch

    from . import autotune
    dev = xs[0].device
    key = "|".join([_device_key(torch, dev), _lib_hash(),
                    signature([x.numel() for x in xs], list(n_maxs), list(precisions))])
    path = cache_path()
    data = _load(path)
    if not refresh and key in data:
        return data[key]["tuning"], {"key": key, "cached": True, "times_ms": data[key]["times_ms"]}
    best, times = autotune(xs, n_maxs, precisions, list(candidates), warmup=warmup, reps=reps)
    data[key] = {"tuning": best, "times_ms": dict(zip(map(json.dumps, candidates), times))}
    try:
        _store(path, data)
    except OSError:
        pass
    return best, {"key": key, "cached": False, "times_ms": data[key]["times_ms"]}
